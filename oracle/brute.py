"""Pure-Python brute force for tiny inputs, used to pin the C oracle (test infrastructure).

Single-precision steps are emulated exactly: every float operation is done in exact rational
arithmetic and then rounded once to the nearest float32 (ties to even), which is what IEEE-754
prescribes for +, -, *, fma and sqrt.  Double steps use Python floats (IEEE doubles, no fusion).
Meant for clouds of at most a few dozen points.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def round_f32(x: Fraction) -> float:
    """Nearest float32 to the exact rational x (ties to even), returned as a Python float."""
    if x == 0:
        return 0.0
    sign = -1 if x < 0 else 1
    a = -x if x < 0 else x
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q_exp = max(e, -126) - 23  # quantum of the float32 grid around a
    q = a / (Fraction(2) ** q_exp)
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    val = Fraction(n) * Fraction(2) ** q_exp
    if val >= Fraction(2) ** 128:
        return sign * math.inf
    return sign * float(val)


def f32(x) -> float:
    return float(np.float32(x))


def sub32(a, b):
    return round_f32(Fraction(a) - Fraction(b))


def mul32(a, b):
    return round_f32(Fraction(a) * Fraction(b))


def fma32(a, b, c):
    return round_f32(Fraction(a) * Fraction(b) + Fraction(c))


def sqrt32(x: float) -> float:
    """Correctly rounded float32 square root of a non-negative float32 value: the candidate c
    whose rounding interval (midpoints to its neighbours) contains sqrt(x), tested exactly by
    squaring the midpoints."""
    fx = Fraction(x)
    if fx == 0:
        return 0.0
    s = np.float32(math.sqrt(x))
    for c in (np.nextafter(s, np.float32(0)), s, np.nextafter(s, np.float32(np.inf))):
        lo = (Fraction(float(np.nextafter(c, np.float32(0)))) + Fraction(float(c))) / 2
        hi = (Fraction(float(c)) + Fraction(float(np.nextafter(c, np.float32(np.inf))))) / 2
        if lo * lo < fx < hi * hi:
            return float(c)
    raise AssertionError("no float32 square-root candidate brackets the input")


# ---------------------------------------------------------------- sampling
def tri_area(p1, p2, p3) -> float:
    e1 = [float(p2[k]) - float(p1[k]) for k in range(3)]
    e2 = [float(p3[k]) - float(p1[k]) for k in range(3)]
    cx = e1[1] * e2[2] - e1[2] * e2[1]
    cy = e1[2] * e2[0] - e1[0] * e2[2]
    cz = e1[0] * e2[1] - e1[1] * e2[0]
    return 0.5 * math.sqrt(cx * cx + cy * cy + cz * cz)


def pick_face(areas, w_lo: int, w_hi: int) -> int:
    cdf = []
    s = 0.0
    for a in areas:
        s = s + a
        cdf.append(s)
    r = float(((w_hi << 32) | w_lo) >> 11) * 2.0 ** -53
    target = r * s
    for k, c in enumerate(cdf):
        if c > target:
            return k
    for k in range(len(areas) - 1, -1, -1):
        if areas[k] > 0:
            return k
    return -1


def barycentric(p1, p2, p3, w_r1: int, w_r2: int):
    r1 = float(w_r1 >> 8) * 2.0 ** -24
    r2 = float(w_r2 >> 8) * 2.0 ** -24
    s = sqrt32(r1)
    u = sub32(1.0, s)
    v = mul32(s, sub32(1.0, r2))
    w = mul32(s, r2)
    x = [fma32(w, f32(p3[k]), fma32(v, f32(p2[k]), mul32(u, f32(p1[k])))) for k in range(3)]
    return x, [u, v, w]


# ---------------------------------------------------------------- Chamfer
def dist32(q, p) -> float:
    dx = sub32(f32(q[0]), f32(p[0]))
    dy = sub32(f32(q[1]), f32(p[1]))
    dz = sub32(f32(q[2]), f32(p[2]))
    return fma32(dz, dz, fma32(dy, dy, mul32(dx, dx)))


def dist_exact(q, p) -> Fraction:
    return sum((Fraction(f32(q[k])) - Fraction(f32(p[k]))) ** 2 for k in range(3))


def nearest(Q, P):
    idx, d32, dex = [], [], []
    for q in Q:
        best, bj = None, -1
        for j, p in enumerate(P):
            d = dist32(q, p)
            if best is None or d < best:
                best, bj = d, j
        idx.append(bj)
        d32.append(best)
        dex.append(dist_exact(q, P[bj]))
    return idx, d32, dex


def chamfer_exact(A, B, reduction=0):
    """Loss of Eq. 1 (reduction 0) or Eq. 2 (reduction 1) as an exact rational, with the
    neighbours decided by the canonical float distance."""
    ia, _, da = nearest(A, B)
    ib, _, db = nearest(B, A)
    if reduction == 1:
        return sum(da, Fraction(0)), ia, ib
    return sum(da, Fraction(0)) / len(A) + sum(db, Fraction(0)) / len(B), ia, ib


def loss_frozen(A, B, ia, ib, reduction=0) -> Fraction:
    """Exact loss with the neighbour indices held fixed (a quadratic in the coordinates)."""
    la = sum((dist_exact(A[i], B[ia[i]]) for i in range(len(A))), Fraction(0))
    if reduction == 1:
        return la
    lb = sum((dist_exact_frac(B[j], A[ib[j]]) for j in range(len(B))), Fraction(0))
    return la / len(A) + lb / len(B)


def dist_exact_frac(q, p) -> Fraction:
    return sum((Fraction(q[k]) - Fraction(p[k])) ** 2 for k in range(3))


def grad_by_exact_differences(A, B, ia, ib, reduction=0):
    """d loss / d A by exact central differences of the frozen-neighbour quadratic: for a
    quadratic the central difference equals the derivative exactly, at any step."""
    h = Fraction(1, 1024)
    g = []
    for i in range(len(A)):
        gi = []
        for k in range(3):
            Ap = [list(map(Fraction, map(f32, a))) for a in A]
            Am = [list(map(Fraction, map(f32, a))) for a in A]
            Ap[i][k] += h
            Am[i][k] -= h
            lp = _loss_frac(Ap, B, ia, ib, reduction)
            lm = _loss_frac(Am, B, ia, ib, reduction)
            gi.append((lp - lm) / (2 * h))
        g.append(gi)
    return g


def _loss_frac(A, B, ia, ib, reduction):
    Bf = [list(map(Fraction, map(f32, b))) for b in B]
    la = sum((dist_exact_frac(A[i], Bf[ia[i]]) for i in range(len(A))), Fraction(0))
    if reduction == 1:
        return la
    lb = sum((dist_exact_frac(Bf[j], A[ib[j]]) for j in range(len(B))), Fraction(0))
    return la / len(A) + lb / len(B)
