"""CPU oracle for the DiffCloud hot path (arXiv 2204.03139, Sec. III, Eq. 1-4).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg are
the only users.  The product library never imports this package, and this package never imports
the product library.  See oracle.c for the arithmetic and the readings it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")

CFLAGS = ["-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-std=c11"]
# DC_ORACLE_SANITIZE=1 builds and loads a separate copy under AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; the Python process must preload libasan)
SANITIZE = os.environ.get("DC_ORACLE_SANITIZE") == "1"
if SANITIZE:
    CFLAGS = CFLAGS + ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                       "-fno-omit-frame-pointer", "-g"]
_SO = os.path.join(_HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (CPU code only)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p
_i = ctypes.c_int


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_SO)
        L.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        L.orc_words_from_seed.argtypes = [ctypes.c_uint64, _i, _i, _u32p]
        L.orc_face_areas.argtypes = [_f32p, _i32p, _i, _i, _f64p]
        L.orc_face_areas.restype = _i
        L.orc_area_cdf.argtypes = [_f64p, _i, _f64p]
        L.orc_area_cdf.restype = _i
        L.orc_pick_face.argtypes = [_f64p, _f64p, _i, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_pick_face.restype = _i
        L.orc_barycentric.argtypes = [_f32p, _f32p, _f32p, ctypes.c_uint32, ctypes.c_uint32,
                                      _f32p, _f32p]
        L.orc_sample_surface.argtypes = [_f32p, _i32p, _i, _i, _i, _i, _u32p, _vp, ctypes.c_long,
                                         _f32p, _i32p, _f32p, _vp, _vp]
        L.orc_sample_surface.restype = _i
        L.orc_rigid_pose.argtypes = [_f64p, _f32p, _i32p, _i, _i, _i, _f64p]
        L.orc_rigid_pose.restype = _i
        L.orc_rigid_pose_grad.argtypes = [_f64p, _f32p, _i32p, _f32p, _i, _i, _i, _f64p, _vp]
        L.orc_rigid_pose_grad.restype = _i
        L.orc_nearest.argtypes = [_f32p, _i, _f32p, _i, _i32p, _f32p, _f64p, _i]
        L.orc_chamfer.argtypes = [_f32p, _f32p, _i, _i, _i, _i, _vp, _i32p, _f32p, _f64p, _i32p,
                                  _f32p, _f64p, _f64p, _i]
        L.orc_chamfer.restype = _i
        L.orc_chamfer_grad.argtypes = [_f32p, _f32p, _i32p, _i32p, _i, _i, _i, _i, _vp, _vp,
                                       _f64p, _vp, _vp, _vp]
        L.orc_chamfer_grad.restype = _i
        L.orc_sample_grad.argtypes = [_f64p, _vp, _i32p, _i32p, _f32p, _i, _i, _i, _i, _f64p, _vp]
        L.orc_sample_grad.restype = _i
        L.orc_points_f64.argtypes = [_f64p, _i32p, _i32p, _f32p, _i, _i, _i, _f64p]
        L.orc_loss_f64.argtypes = [_f64p, _f32p, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _i]
        L.orc_loss_f64.restype = ctypes.c_double
        L.orc_max_threads.restype = _i
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _c(x, dt):
    return np.ascontiguousarray(x, dtype=dt)


def _ptr(x):
    return None if x is None else x.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return lib().orc_max_threads()


# ------------------------------------------------------------------ random words
def philox4x64_10(counter, key):
    """One Philox4x64-10 block (Salmon et al., SC'11): 4 x uint64 counter, 2 x uint64 key."""
    c = _c(counter, np.uint64)
    k = _c(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(c, k, out)
    return out


def words_from_seed(seed: int, T: int, N: int) -> np.ndarray:
    out = np.zeros((T, N, 4), np.uint32)
    lib().orc_words_from_seed(ctypes.c_uint64(seed & (2**64 - 1)), T, N, out)
    return out


# ------------------------------------------------------------------ sampling (Sec. III-B)
def face_areas(verts_frame, faces) -> np.ndarray:
    v = _c(verts_frame, np.float32)
    f = _c(faces, np.int32)
    out = np.zeros(f.shape[0], np.float64)
    rc = lib().orc_face_areas(v, f, v.shape[0], f.shape[0], out)
    if rc != 0:
        raise OracleError(f"face_areas: status {rc}")
    return out


def area_cdf(areas):
    a = _c(areas, np.float64)
    out = np.zeros_like(a)
    rc = lib().orc_area_cdf(a, a.shape[0], out)
    return out, rc


def pick_face(areas, cdf, w_lo: int, w_hi: int) -> int:
    return lib().orc_pick_face(_c(areas, np.float64), _c(cdf, np.float64), len(areas),
                               ctypes.c_uint32(w_lo), ctypes.c_uint32(w_hi))


def barycentric(p1, p2, p3, w_r1: int, w_r2: int):
    x = np.zeros(3, np.float32)
    b = np.zeros(3, np.float32)
    lib().orc_barycentric(_c(p1, np.float32), _c(p2, np.float32), _c(p3, np.float32),
                          ctypes.c_uint32(w_r1), ctypes.c_uint32(w_r2), x, b)
    return x, b


def sample_surface(verts, faces, N: int, words=None, seed: int | None = None,
                   return_cdf: bool = False, face_mask=None):
    """Area-weighted sampling of N points per frame: returns points, face_idx, bary.
    face_mask (optional, [F] or [T,F], nonzero = may be drawn) restricts the draws to a subset of
    faces, each keeping its area weight (Sec. IV: occlusion heuristic, cloth-only clouds)."""
    v = _c(verts, np.float32)
    if v.ndim == 2:
        v = v[None]
    T, V, _ = v.shape
    f = _c(faces, np.int32)
    F = f.shape[0]
    if words is None:
        words = words_from_seed(seed, T, N)
    w = _c(words, np.uint32).reshape(T, N, 4)
    pts = np.zeros((T, N, 3), np.float32)
    fi = np.zeros((T, N), np.int32)
    ba = np.zeros((T, N, 3), np.float32)
    A = np.zeros((T, F), np.float64)
    C = np.zeros((T, F), np.float64)
    m, stride = None, 0
    if face_mask is not None:
        m = np.ascontiguousarray(face_mask, np.uint8)
        if m.shape not in ((F,), (T, F)):
            raise ValueError("face_mask must be [F] or [T,F]")
        stride = F if m.ndim == 2 else 0
    rc = lib().orc_sample_surface(v, f, T, V, F, N, w, _ptr(m), stride, pts, fi, ba, _ptr(A),
                                  _ptr(C))
    if rc != 0:
        raise OracleError(f"sample_surface: status {rc}")
    if return_cdf:
        return pts, fi, ba, A, C
    return pts, fi, ba


# ------------------------------------------------------------------ Chamfer (Sec. III-A)
def nearest(Q, P, nthreads: int = 0):
    q = _c(Q, np.float32)
    p = _c(P, np.float32)
    n = q.shape[0]
    idx = np.zeros(n, np.int32)
    d32 = np.zeros(n, np.float32)
    d64 = np.zeros(n, np.float64)
    lib().orc_nearest(q, n, p, p.shape[0], idx, d32, d64, nthreads)
    return idx, d32, d64


def chamfer(a, b, reduction: int = 0, frame_w=None, nthreads: int = 0):
    """Eq. 1 (reduction 0) or Eq. 2 (reduction 1) per frame; returns dict of outputs."""
    A = _c(a, np.float32)
    B = _c(b, np.float32)
    if A.ndim == 2:
        A, B = A[None], B[None]
    T, Na, _ = A.shape
    Nb = B.shape[1]
    fw = None if frame_w is None else _c(frame_w, np.float32)
    out = dict(idx_a=np.zeros((T, Na), np.int32), d32a=np.zeros((T, Na), np.float32),
               d64a=np.zeros((T, Na), np.float64), idx_b=np.zeros((T, Nb), np.int32),
               d32b=np.zeros((T, Nb), np.float32), d64b=np.zeros((T, Nb), np.float64),
               loss=np.zeros(T, np.float64))
    rc = lib().orc_chamfer(A, B, T, Na, Nb, reduction, _ptr(fw), out["idx_a"], out["d32a"],
                           out["d64a"], out["idx_b"], out["d32b"], out["d64b"], out["loss"],
                           nthreads)
    if rc != 0:
        raise OracleError(f"chamfer: status {rc}")
    return out


def chamfer_grad(a, b, idx_a, idx_b, reduction: int = 0, frame_w=None, grad_loss=None,
                 want_b: bool = False):
    A = _c(a, np.float32)
    B = _c(b, np.float32)
    if A.ndim == 2:
        A, B = A[None], B[None]
    T, Na, _ = A.shape
    Nb = B.shape[1]
    ia = _c(idx_a, np.int32).reshape(T, Na)
    ib = _c(idx_b, np.int32).reshape(T, Nb)
    fw = None if frame_w is None else _c(frame_w, np.float32)
    gl = None if grad_loss is None else _c(grad_loss, np.float64)
    ga = np.zeros((T, Na, 3), np.float64)
    gaa = np.zeros((T, Na, 3), np.float64)
    gb = np.zeros((T, Nb, 3), np.float64) if want_b else None
    gba = np.zeros((T, Nb, 3), np.float64) if want_b else None
    rc = lib().orc_chamfer_grad(A, B, ia, ib, T, Na, Nb, reduction, _ptr(fw), _ptr(gl), ga,
                                _ptr(gaa), _ptr(gb), _ptr(gba))
    if rc != 0:
        raise OracleError(f"chamfer_grad: status {rc}")
    return dict(ga=ga, ga_abs=gaa, gb=gb, gb_abs=gba)


def sample_grad(gpoints, faces, face_idx, bary, V: int, gpoints_abs=None):
    g = _c(gpoints, np.float64)
    T, N, _ = g.shape
    f = _c(faces, np.int32)
    gabs = None if gpoints_abs is None else _c(gpoints_abs, np.float64)
    gv = np.zeros((T, V, 3), np.float64)
    gva = np.zeros((T, V, 3), np.float64)
    rc = lib().orc_sample_grad(g, _ptr(gabs), f, _c(face_idx, np.int32), _c(bary, np.float32),
                               T, V, f.shape[0], N, gv, _ptr(gva))
    if rc != 0:
        raise OracleError(f"sample_grad: status {rc}")
    return gv, gva


def points_f64(verts64, faces, face_idx, bary):
    v = _c(verts64, np.float64)
    T, V, _ = v.shape
    N = face_idx.shape[1]
    out = np.zeros((T, N, 3), np.float64)
    lib().orc_points_f64(v, _c(faces, np.int32), _c(face_idx, np.int32), _c(bary, np.float32),
                         T, V, N, out)
    return out


def loss_f64(points64, b, reduction: int = 0, frame_w=None, idx_a=None, idx_b=None,
             return_idx: bool = False, nthreads: int = 0):
    p = _c(points64, np.float64)
    B = _c(b, np.float32)
    T, Na, _ = p.shape
    Nb = B.shape[1]
    fw = None if frame_w is None else _c(frame_w, np.float32)
    ia = None if idx_a is None else _c(idx_a, np.int32)
    ib = None if idx_b is None else _c(idx_b, np.int32)
    oa = np.zeros((T, Na), np.int32) if return_idx else None
    ob = np.zeros((T, Nb), np.int32) if return_idx else None
    val = lib().orc_loss_f64(p, B, T, Na, Nb, reduction, _ptr(fw), _ptr(ia), _ptr(ib), _ptr(oa),
                             _ptr(ob), nthreads)
    if return_idx:
        return val, oa, ob
    return val


def full_gradient(verts, faces, observed, face_idx, bary, points, reduction=0, frame_w=None,
                  grad_loss=None):
    """Vertex gradient of sum_t loss[t]: Chamfer gradient through Eq. 4, plus its abs-sum."""
    ch = chamfer(points, observed, reduction, frame_w)
    g = chamfer_grad(points, observed, ch["idx_a"], ch["idx_b"], reduction, frame_w, grad_loss)
    V = np.asarray(verts).shape[-2]
    gv, gva = sample_grad(g["ga"], faces, face_idx, bary, V, g["ga_abs"])
    return gv, gva, ch


def fd_gradient(verts, faces, observed, face_idx, bary, coords, h=1e-4, reduction=0,
                frame_w=None):
    """Central differences (L(V+h e_k) - L(V-h e_k)) / 2h in double for the listed
    (frame, vertex, axis) coordinates, face choice and weights fixed.  A vertex of frame t only
    moves frame t's points, so only that frame's term of the loss is differenced.  Returns
    (fd, frozen_fd, moved): moved flags coordinates whose neighbours changed between V-h and V+h,
    and frozen_fd repeats the difference with the neighbours at V held fixed."""
    V64 = np.asarray(verts, dtype=np.float64).copy()
    if V64.ndim == 2:
        V64 = V64[None]
    obs = np.asarray(observed, dtype=np.float32)
    fw = None if frame_w is None else np.asarray(frame_w, np.float32)
    fd = np.zeros(len(coords))
    fdz = np.zeros(len(coords))
    moved = np.zeros(len(coords), bool)
    base = {}
    for n, (t, v, k) in enumerate(coords):
        sl = slice(t, t + 1)
        fwt = None if fw is None else fw[sl]
        if t not in base:
            p0 = points_f64(V64[sl], faces, face_idx[sl], bary[sl])
            _, ia0, ib0 = loss_f64(p0, obs[sl], reduction, fwt, return_idx=True)
            base[t] = (ia0, ib0)
        ia0, ib0 = base[t]
        old = V64[t, v, k]
        V64[t, v, k] = old + h
        pp = points_f64(V64[sl], faces, face_idx[sl], bary[sl])
        lp, iap, ibp = loss_f64(pp, obs[sl], reduction, fwt, return_idx=True)
        lpz = loss_f64(pp, obs[sl], reduction, fwt, idx_a=ia0, idx_b=ib0)
        V64[t, v, k] = old - h
        pm = points_f64(V64[sl], faces, face_idx[sl], bary[sl])
        lm, iam, ibm = loss_f64(pm, obs[sl], reduction, fwt, return_idx=True)
        lmz = loss_f64(pm, obs[sl], reduction, fwt, idx_a=ia0, idx_b=ib0)
        V64[t, v, k] = old
        fd[n] = (lp - lm) / (2 * h)
        fdz[n] = (lpz - lmz) / (2 * h)
        moved[n] = not (np.array_equal(iap, iam) and np.array_equal(ibp, ibm))
    return fd, fdz, moved


# ------------------------------------------------------------------ rigid bodies (Sec. III-C)
def rigid_pose(q, p0, body_start, V: int | None = None):
    """Vertices [T,V,3] (double) of rigid bodies at poses q [T,B,6] = (t, phi, theta, psi):
    p = Rz(psi) Ry(theta) Rx(phi) p0 + t for the vertices [body_start[b], body_start[b+1])."""
    qq = _c(q, np.float64)
    T, B, _ = qq.shape
    pp = _c(p0, np.float32)
    V = pp.shape[0] if V is None else V
    out = np.zeros((T, V, 3), np.float64)
    rc = lib().orc_rigid_pose(qq, pp, _c(body_start, np.int32), T, B, V, out)
    if rc != 0:
        raise OracleError(f"rigid_pose: status {rc}")
    return out


def rigid_pose_grad(q, p0, body_start, grad_verts):
    """Pose gradient [T,B,6] = sum over each body's vertices of J^T g, and its abs-sum."""
    qq = _c(q, np.float64)
    T, B, _ = qq.shape
    g = _c(grad_verts, np.float32)
    V = g.shape[1]
    gq = np.zeros((T, B, 6), np.float64)
    ga = np.zeros((T, B, 6), np.float64)
    rc = lib().orc_rigid_pose_grad(qq, _c(p0, np.float32), _c(body_start, np.int32), g, T, B, V,
                                   gq, _ptr(ga))
    if rc != 0:
        raise OracleError(f"rigid_pose_grad: status {rc}")
    return gq, ga
