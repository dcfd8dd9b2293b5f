"""Seeded synthetic inputs: cloth-like mesh trajectories, observed clouds, sampler words.

Recipe (the simulator of the paper is not rebuilt; these trajectories stand in for its output):

* Mesh: an n x n vertex grid over [-0.5, 0.5]^2 m.  Vertex (i, j) sits at
  x = -0.5 + i/(n-1), y = -0.5 + j/(n-1) and has index v = j*n + i.  Each grid quad is split
  along its (i, j) -> (i+1, j+1) diagonal into two counter-clockwise triangles, so F = 2 (n-1)^2.
* Motion: only z moves.  z(x, y, t) = sum_{k=1..3} amp_k sin(2 pi (kx_k x + ky_k y) + phi_k
  + omega_k t) - sag * (t / (T-1)) * (1 - 4x^2)(1 - 4y^2), with amp_k = 0.05,
  kx, ky ~ U(-3, 3) cycles/m, phi ~ U(0, 2 pi), omega ~ U(0.05, 0.2) rad/frame.  |z| <= 0.27.
* Observed cloud: the "perturbed" surface uses phi_k + U(-0.3, 0.3), amp_k * U(0.9, 1.1) and
  sag * 1.2 (the single-frame workload uses the unperturbed mesh).  Points are spread uniformly
  over the area of the piecewise-linear mesh surface by rejection in the (x, y) square: a uniform
  (x, y) is kept with probability J / J_max, where J = sqrt(1 + z_x^2 + z_y^2) is the area element
  of the grid triangle under it (its area over its projected area) and J_max the frame's largest,
  then lifted onto the surface (a height-field lookup) and moved by i.i.d. N(0, 0.005^2) noise per
  axis.  This is input data, generated here in float64 and handed to every consumer in float32.
* Sampler words: four uint32 per (frame, point), drawn from numpy's generator.

Every stream is seeded from (workload id, stream id), so inputs are reproducible.
"""
from __future__ import annotations

import math

import numpy as np

# stream ids inside one workload's seed space
S_MESH, S_SIM_WORDS, S_OBS_PERTURB, S_OBS_XY, S_NOISE, S_FD, S_REQ, S_ARRIVAL = range(8)

CONFIGS = {
    1: dict(name="fp32-single-frame 25x25 grid, 2048 vs 2048 points, 1 frame",
            n=25, T=1, Na=2048, Nb=2048, sag=0.0, same_mesh=True),
    2: dict(name="fp32-trajectory 50x50 grid, 8192 vs 8192 points, 40 frames",
            n=50, T=40, Na=8192, Nb=8192, sag=0.1, same_mesh=False),
    3: dict(name="autograd 25x25 grid, 2048 vs 2048 points, 4 frames",
            n=25, T=4, Na=2048, Nb=2048, sag=0.1, same_mesh=False),
    4: dict(name="precision 100x100 grid, 65536 vs 65536 points, 100 frames",
            n=100, T=100, Na=65536, Nb=65536, sag=0.1, same_mesh=False),
    5: dict(name="serving 256 requests, grids 10..80, points 512..32768, 1..60 frames",
            n_requests=256, rate_hz=200.0, budget_bytes=64 << 30),
}


def _rng(cfg_id: int, stream: int, extra: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg_id), int(stream), int(extra)]))


def grid_mesh(n: int):
    """Return (xy [V,2] float64, faces [F,3] int32) for the n x n grid described above."""
    if n < 2:
        raise ValueError("grid needs n >= 2")
    lin = -0.5 + np.arange(n, dtype=np.float64) / (n - 1)
    X, Y = np.meshgrid(lin, lin, indexing="xy")  # X[j, i] = lin[i], Y[j, i] = lin[j]
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    i = np.arange(n - 1)
    I, J = np.meshgrid(i, i, indexing="xy")
    v00 = (J * n + I).ravel()
    v10 = v00 + 1
    v01 = v00 + n
    v11 = v00 + n + 1
    tri1 = np.stack([v00, v10, v11], axis=1)
    tri2 = np.stack([v00, v11, v01], axis=1)
    faces = np.empty((2 * len(v00), 3), dtype=np.int32)
    faces[0::2] = tri1
    faces[1::2] = tri2
    return xy, faces


def _surface_params(cfg_id: int, extra: int = 0):
    r = _rng(cfg_id, S_MESH, extra)
    return dict(
        amp=np.full(3, 0.05),
        kx=r.uniform(-3.0, 3.0, 3),
        ky=r.uniform(-3.0, 3.0, 3),
        phi=r.uniform(0.0, 2 * math.pi, 3),
        omega=r.uniform(0.05, 0.2, 3),
    )


def _perturb(p: dict, cfg_id: int, extra: int = 0) -> dict:
    r = _rng(cfg_id, S_OBS_PERTURB, extra)
    q = dict(p)
    q["phi"] = p["phi"] + r.uniform(-0.3, 0.3, 3)
    q["amp"] = p["amp"] * r.uniform(0.9, 1.1, 3)
    return q


def _height(p: dict, x, y, t: float, T: int, sag: float):
    z = np.zeros(np.broadcast(x, y).shape, dtype=np.float64)
    for k in range(3):
        z += p["amp"][k] * np.sin(2 * math.pi * (p["kx"][k] * x + p["ky"][k] * y)
                                  + p["phi"][k] + p["omega"][k] * t)
    if T > 1 and sag != 0.0:
        z -= sag * (t / (T - 1)) * (1 - 4 * x * x) * (1 - 4 * y * y)
    return z


def trajectory(n: int, T: int, cfg_id: int, sag: float = 0.1, extra: int = 0,
               perturbed: bool = False):
    """Vertex trajectory [T, V, 3] float32 and faces [F, 3] int32 for the grid cloth."""
    xy, faces = grid_mesh(n)
    p = _surface_params(cfg_id, extra)
    if perturbed:
        p = _perturb(p, cfg_id, extra)
        sag = sag * 1.2
    V = xy.shape[0]
    verts = np.empty((T, V, 3), dtype=np.float64)
    for t in range(T):
        verts[t, :, 0] = xy[:, 0]
        verts[t, :, 1] = xy[:, 1]
        verts[t, :, 2] = _height(p, xy[:, 0], xy[:, 1], float(t), T, sag)
    return verts.astype(np.float32), faces


def _grid_cell(zgrid: np.ndarray, n: int, x: np.ndarray, y: np.ndarray):
    """Height of the piecewise-linear grid surface at (x, y) (height-field lookup) and the area
    element sqrt(1 + z_x^2 + z_y^2) of the grid triangle under (x, y)."""
    gx = (x + 0.5) * (n - 1)
    gy = (y + 0.5) * (n - 1)
    i = np.clip(np.floor(gx).astype(np.int64), 0, n - 2)
    j = np.clip(np.floor(gy).astype(np.int64), 0, n - 2)
    s = gx - i
    r = gy - j
    z00 = zgrid[j, i]
    z10 = zgrid[j, i + 1]
    z01 = zgrid[j + 1, i]
    z11 = zgrid[j + 1, i + 1]
    # lower triangle (v00, v10, v11) when s >= r, upper (v00, v11, v01) otherwise
    lower = s >= r
    z_lo = z00 + s * (z10 - z00) + r * (z11 - z10)
    z_up = z00 + r * (z01 - z00) + s * (z11 - z01)
    # slopes in metres per metre: one grid step is 1 / (n - 1)
    zx = np.where(lower, z10 - z00, z11 - z01) * (n - 1)
    zy = np.where(lower, z11 - z10, z01 - z00) * (n - 1)
    return np.where(lower, z_lo, z_up), np.sqrt(1.0 + zx * zx + zy * zy)


def _area_element_max(zgrid: np.ndarray, n: int) -> float:
    """Largest area element over all triangles of the grid surface."""
    z00, z10 = zgrid[:-1, :-1], zgrid[:-1, 1:]
    z01, z11 = zgrid[1:, :-1], zgrid[1:, 1:]
    lo = (z10 - z00) ** 2 + (z11 - z10) ** 2
    up = (z11 - z01) ** 2 + (z01 - z00) ** 2
    return float(np.sqrt(1.0 + max(lo.max(), up.max()) * (n - 1) ** 2))


def _surface_uniform_xy(rxy: np.random.Generator, zgrid: np.ndarray, n: int, count: int):
    """`count` points spread uniformly over the area of the grid surface: uniform (x, y) kept
    with probability J / J_max (rejection), in the order they are drawn; returns x, y, z."""
    jmax = _area_element_max(zgrid, n)
    xs, ys, zs = [], [], []
    have = 0
    while have < count:
        m = max(1024, int((count - have) * 1.25 * jmax))
        x = rxy.uniform(-0.5, 0.5, m)
        y = rxy.uniform(-0.5, 0.5, m)
        keep_u = rxy.uniform(0.0, 1.0, m)
        z, jac = _grid_cell(zgrid, n, x, y)
        keep = keep_u * jmax < jac
        xs.append(x[keep])
        ys.append(y[keep])
        zs.append(z[keep])
        have += int(keep.sum())
    return (np.concatenate(xs)[:count], np.concatenate(ys)[:count],
            np.concatenate(zs)[:count])


def observed_cloud(n: int, T: int, Nb: int, cfg_id: int, sag: float = 0.1,
                   same_mesh: bool = False, sigma: float = 0.005, extra: int = 0):
    """Observed cloud [T, Nb, 3] float32: points on the (perturbed) mesh plus Gaussian noise."""
    verts, _ = trajectory(n, T, cfg_id, sag=sag, extra=extra, perturbed=not same_mesh)
    rxy = _rng(cfg_id, S_OBS_XY, extra)
    rn = _rng(cfg_id, S_NOISE, extra)
    out = np.empty((T, Nb, 3), dtype=np.float64)
    for t in range(T):
        zgrid = verts[t, :, 2].astype(np.float64).reshape(n, n)
        x, y, z = _surface_uniform_xy(rxy, zgrid, n, Nb)
        out[t, :, 0] = x
        out[t, :, 1] = y
        out[t, :, 2] = z
        out[t] += rn.normal(0.0, sigma, (Nb, 3))
    return out.astype(np.float32)


def sim_uniform_words(T: int, N: int, cfg_id: int, extra: int = 0) -> np.ndarray:
    """Four uint32 random words per (frame, point): [T, N, 4]."""
    r = _rng(cfg_id, S_SIM_WORDS, extra)
    return r.integers(0, 2**32, size=(T, N, 4), dtype=np.uint64).astype(np.uint32)


def fd_vertices(V: int, count: int, cfg_id: int) -> np.ndarray:
    r = _rng(cfg_id, S_FD)
    return np.sort(r.choice(V, size=min(count, V), replace=False)).astype(np.int64)


def workload(cfg_id: int, T: int | None = None):
    """Inputs of one fixed workload: dict with verts, faces, observed, words and sizes."""
    c = CONFIGS[cfg_id]
    T = c["T"] if T is None else T
    verts, faces = trajectory(c["n"], T, cfg_id, sag=c["sag"])
    obs = observed_cloud(c["n"], T, c["Nb"], cfg_id, sag=c["sag"], same_mesh=c["same_mesh"])
    words = sim_uniform_words(T, c["Na"], cfg_id)
    return dict(verts=verts, faces=faces, observed=obs, words=words, T=T, V=verts.shape[1],
                F=faces.shape[0], Na=c["Na"], Nb=c["Nb"], seed=1000 + cfg_id, name=c["name"])


def serving_requests(cfg_id: int = 5, n_requests: int | None = None, rate_hz: float | None = None,
                     arrival_seed: int = 0, max_grid: int = 80, max_points: int = 32768,
                     max_frames: int = 60):
    """Request mix for the serving loop: list of dicts plus Poisson arrival offsets (s)."""
    c = CONFIGS[5]
    nreq = c["n_requests"] if n_requests is None else n_requests
    rate = c["rate_hz"] if rate_hz is None else rate_hz
    r = _rng(cfg_id, S_REQ)
    ra = _rng(cfg_id, S_ARRIVAL, arrival_seed)
    reqs = []
    for k in range(nreq):
        n = int(r.integers(10, max_grid + 1))
        na = int(round(math.exp(r.uniform(math.log(512), math.log(max_points)))))
        nb = int(round(math.exp(r.uniform(math.log(512), math.log(max_points)))))
        T = int(r.integers(1, max_frames + 1))
        reqs.append(dict(n=n, Na=na, Nb=nb, T=T, seed=10_000 + k, extra=k))
    gaps = ra.exponential(1.0 / rate, nreq)
    arrivals = np.cumsum(gaps) - gaps[0]
    return reqs, arrivals


def request_inputs(req: dict, cfg_id: int = 5):
    verts, faces = trajectory(req["n"], req["T"], cfg_id, sag=0.1, extra=req["extra"])
    obs = observed_cloud(req["n"], req["T"], req["Nb"], cfg_id, sag=0.1, extra=req["extra"])
    return verts, faces, obs
