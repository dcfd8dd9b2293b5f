"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the same seeded
inputs.  Indices and sampled points must match bit for bit; distances, losses and gradients to
the tolerances stated in each test (1e-5 relative in float32)."""
import numpy as np
import pytest

import oracle
from workloads import gen

from gpu_helpers import assert_grad, assert_rel, dev, gpu, host, say, torch

pytestmark = pytest.mark.gpu


def _sample_both(p, verts, faces, N, words=None, seed=None):
    """GPU and oracle sampling of the same trajectory."""
    vt, ft = dev(verts), dev(faces)
    if words is not None:
        g = p.sample_surface(vt, ft, N, uniforms=dev(words.view(np.int32)))
        o = oracle.sample_surface(verts, faces, N, words=words)
    else:
        g = p.sample_surface(vt, ft, N, seed=seed)
        o = oracle.sample_surface(verts, faces, N, seed=seed)
    torch.cuda.synchronize()
    return [host(x) for x in g], o


@pytest.mark.parametrize("case", ["cfg1-words", "cfg1-philox", "cfg2-3frames", "ragged"])
def test_sample_parity(case):
    p = gpu()
    say(f"[sample] {case}")
    if case.startswith("cfg1"):
        w = gen.workload(1)
        verts, faces, N = w["verts"], w["faces"], w["Na"]
        words = w["words"] if case.endswith("words") else None
        seed = None if words is not None else w["seed"]
    elif case == "cfg2-3frames":
        w = gen.workload(2, T=3)
        verts, faces, N, words, seed = w["verts"], w["faces"], w["Na"], w["words"], None
    else:  # tiny mesh, ragged point count
        verts, faces = gen.trajectory(3, 2, 9)
        N, words, seed = 37, None, 123456789012345
    (gp, gf, gb), (op, of, ob) = _sample_both(p, verts, faces, N, words, seed)
    assert np.array_equal(gf, of)
    assert np.array_equal(gp.view(np.uint32), op.view(np.uint32))
    assert np.array_equal(gb.view(np.uint32), ob.view(np.uint32))


@pytest.mark.parametrize("mode", ["shared-upper-half", "per-frame-runs", "philox-shared"])
def test_masked_sample_parity(mode):
    """Subset sampling: points, weights and faces bit-exact against the oracle with the same mask;
    no point lands on an excluded face."""
    p = gpu()
    say(f"[sample] masked {mode}")
    w = gen.workload(2, T=3)
    verts, faces, N = w["verts"], w["faces"], w["Na"]
    F = len(faces)
    if mode == "per-frame-runs":  # runs of 37 consecutive excluded faces, shifted per frame
        mask = np.stack([((np.arange(F) + 11 * t) // 37) % 2 for t in range(3)]).astype(np.uint8)
    else:  # the upper half of the cloth, as in the occlusion heuristic of the fold scenario
        mask = (verts[0][faces][:, :, 1].mean(axis=1) > 0).astype(np.uint8)
    words = None if mode == "philox-shared" else w["words"]
    vt, ft = dev(verts), dev(faces)
    m = torch.from_numpy(mask).to("cuda")
    if words is None:
        g = p.sample_surface(vt, ft, N, seed=w["seed"], face_mask=m)
        o = oracle.sample_surface(verts, faces, N, seed=w["seed"], face_mask=mask)
    else:
        g = p.sample_surface(vt, ft, N, uniforms=dev(words.view(np.int32)), face_mask=m)
        o = oracle.sample_surface(verts, faces, N, words=words, face_mask=mask)
    gp, gf, gb = (host(x) for x in g)
    assert np.array_equal(gf, o[1])
    assert np.array_equal(gp.view(np.uint32), o[0].view(np.uint32))
    assert np.array_equal(gb.view(np.uint32), o[2].view(np.uint32))
    rows = mask if mask.ndim == 2 else np.broadcast_to(mask, (3, F))
    assert all(np.all(rows[t][gf[t]] == 1) for t in range(3))


def test_masked_sample_empty_subset_and_arguments():
    p = gpu()
    ctx = p.Context(0)
    verts, faces = gen.trajectory(6, 2, 3)
    F = len(faces)
    mask = np.ones((2, F), np.uint8)
    mask[1] = 0  # frame 1 has nothing to draw from
    pts, fi, _ = p.sample_surface(dev(verts), dev(faces), 16, seed=3, ctx=ctx,
                                  face_mask=torch.from_numpy(mask).to("cuda"))
    with pytest.raises(p.DCError) as e:
        ctx.sync()
    assert e.value.code == -5
    fi = host(fi)
    assert np.all(fi[1] == -1) and np.all(fi[0] >= 0)
    with pytest.raises(ValueError):  # wrong mask shape
        p.sample_surface(dev(verts), dev(faces), 16, ctx=ctx,
                         face_mask=torch.ones(F + 1, dtype=torch.uint8, device="cuda"))
    ctx.close()


def test_sqrt_all_levels():
    """Every one of the 2^24 values of r1 goes through a correctly rounded square root: with
    r2 = 0 the weight v equals s = sqrt(r1) exactly, compared with the host's IEEE sqrt."""
    p = gpu()
    say("[sample] sqrt over 2^24 levels")
    n = 1 << 24
    verts = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32)
    faces = np.array([[0, 1, 2]], np.int32)
    words = np.zeros((1, n, 4), np.uint32)
    words[0, :, 2] = np.arange(n, dtype=np.uint32) << 8
    _, _, b = p.sample_surface(dev(verts), dev(faces), n, uniforms=dev(words.view(np.int32)))
    s_gpu = host(b)[0, :, 1]
    r1 = (np.arange(n, dtype=np.float64) * 2.0**-24).astype(np.float32)
    s_host = np.sqrt(r1)
    assert np.array_equal(s_gpu.view(np.uint32), s_host.view(np.uint32))


def test_sample_degenerate_and_bad_faces():
    p = gpu()
    say("[sample] degenerate / bad faces")
    ctx = p.Context(0)
    verts = np.zeros((2, 3, 3), np.float32)
    verts[1] = [[0, 0, 0], [1, 0, 0], [0, 1, 0]]  # frame 1 fine, frame 0 zero area
    faces = np.array([[0, 1, 2]], np.int32)
    pts, fi, ba = p.sample_surface(dev(verts), dev(faces), 5, seed=1, ctx=ctx)
    with pytest.raises(p.DCError) as e:
        ctx.sync()
    assert e.value.code == -5
    fi = host(fi)
    assert np.all(fi[0] == -1) and np.all(fi[1] == 0)
    assert np.all(np.isnan(host(pts)[0]))
    ctx.sync()  # the status is cleared after being reported
    bad = np.array([[0, 1, 7]], np.int32)
    p.sample_surface(dev(verts[1:]), dev(bad), 5, seed=1, ctx=ctx)
    with pytest.raises(p.DCError) as e:
        ctx.sync()
    assert e.value.code == -1
    ctx.close()


def test_invalid_arguments():
    p = gpu()
    a = torch.zeros((1, 4, 3), device="cuda")
    with pytest.raises(p.DCError) as e:
        p.chamfer_fwd(a, a, precision=7)
    assert e.value.code == -1
    with pytest.raises(p.DCError):
        p.chamfer_fwd(a, a, reduction=3)
    z = torch.zeros((1, 0, 3), device="cuda")
    with pytest.raises(p.DCError):
        p.chamfer_fwd(z, a)
    with pytest.raises(ValueError):
        p.chamfer_fwd(a[:, ::2], a)


def _chamfer_both(p, A, B, reduction=0, frame_w=None, precision=0):
    g = p.chamfer_fwd(dev(A), dev(B), precision=precision, reduction=reduction,
                      frame_w=None if frame_w is None else dev(frame_w))
    torch.cuda.synchronize()
    g = {k: host(v) for k, v in g.items()}
    o = oracle.chamfer(A, B, reduction, frame_w)
    return g, o


def _check_chamfer(g, o):
    assert np.array_equal(g["idx_a"], o["idx_a"])
    assert np.array_equal(g["idx_b"], o["idx_b"])
    assert np.array_equal(g["dist_a"].view(np.uint32), o["d32a"].view(np.uint32))
    assert np.array_equal(g["dist_b"].view(np.uint32), o["d32b"].view(np.uint32))
    nz = o["d64a"] > 0
    assert_rel(g["dist_a"][nz], o["d64a"][nz], 1e-5, "dist_a vs double")
    nz = o["d64b"] > 0
    assert_rel(g["dist_b"][nz], o["d64b"][nz], 1e-5, "dist_b vs double")
    assert_rel(g["loss"], o["loss"], 1e-5, "loss")


CHAMFER_CASES = {
    "cfg1": lambda: (lambda w: (oracle.sample_surface(w["verts"], w["faces"], w["Na"],
                                                      words=w["words"])[0], w["observed"]))(
        gen.workload(1)),
    "cfg2-3frames": lambda: (lambda w: (oracle.sample_surface(w["verts"], w["faces"], w["Na"],
                                                              words=w["words"])[0],
                                        w["observed"]))(gen.workload(2, T=3)),
    "ragged-1x1": lambda: (np.random.default_rng(1).uniform(-.5, .5, (2, 1, 3)).astype(np.float32),
                           np.random.default_rng(2).uniform(-.5, .5, (2, 1, 3)).astype(np.float32)),
    "ragged-1000x4097": lambda: (
        np.random.default_rng(3).uniform(-.5, .5, (2, 1000, 3)).astype(np.float32),
        np.random.default_rng(4).uniform(-.5, .5, (2, 4097, 3)).astype(np.float32)),
    "ragged-1025x3": lambda: (
        np.random.default_rng(5).uniform(-.5, .5, (1, 1025, 3)).astype(np.float32),
        np.random.default_rng(6).uniform(-.5, .5, (1, 3, 3)).astype(np.float32)),
    "tall-70000x5": lambda: (
        np.random.default_rng(9).uniform(-.5, .5, (2, 70000, 3)).astype(np.float32),
        np.random.default_rng(10).uniform(-.5, .5, (2, 5, 3)).astype(np.float32)),
    "wide-3x70000": lambda: (
        np.random.default_rng(11).uniform(-.5, .5, (2, 3, 3)).astype(np.float32),
        np.random.default_rng(12).uniform(-.5, .5, (2, 70000, 3)).astype(np.float32)),
    "frames-500x300x257": lambda: (
        np.random.default_rng(13).uniform(-.5, .5, (500, 300, 3)).astype(np.float32),
        np.random.default_rng(14).uniform(-.5, .5, (500, 257, 3)).astype(np.float32)),
    "slices-2x20000": lambda: (
        np.random.default_rng(7).uniform(-.5, .5, (1, 20000, 3)).astype(np.float32),
        np.random.default_rng(8).uniform(-.5, .5, (1, 20000, 3)).astype(np.float32)),
}


@pytest.mark.parametrize("case", list(CHAMFER_CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_chamfer_parity(case, precision):
    p = gpu()
    say(f"[chamfer] {case} precision={precision}")
    A, B = CHAMFER_CASES[case]()
    g, o = _chamfer_both(p, A, B, precision=precision)
    _check_chamfer(g, o)


@pytest.mark.parametrize("precision", [0, 1])
def test_chamfer_ties_and_identity(precision):
    p = gpu()
    say(f"[chamfer] ties precision={precision}")
    r = np.random.default_rng(21)
    A = r.uniform(-.5, .5, (1, 3000, 3)).astype(np.float32)
    g, o = _chamfer_both(p, A, A.copy(), precision=precision)
    _check_chamfer(g, o)
    assert np.array_equal(g["idx_a"][0], np.arange(3000)) and g["loss"][0] == 0.0
    # exact duplicates in the target: ties must go to the smallest index
    B = np.concatenate([A[:, :1500], A[:, :1500], A[:, 1500:]], axis=1)
    g, o = _chamfer_both(p, A, B, precision=precision)
    _check_chamfer(g, o)
    # a grid with many equidistant neighbours
    x = np.arange(16, dtype=np.float32) / 16
    G = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(1, -1, 3)
    Q = (G[:, ::7] + np.float32(1 / 32)).astype(np.float32)
    g, o = _chamfer_both(p, Q, G, precision=precision)
    _check_chamfer(g, o)


# query rows per workgroup of the two-direction screen (the column partials are per workgroup):
# four waves of eight 16-row tiles
WG_ROWS = 512


def _periodic_rows(n_rows, period=37, seed=41):
    """Rows repeating `period` points: every row workgroup holds the same points, so each target's
    column partials tie exactly across all workgroups."""
    r = np.random.default_rng(seed)
    P = r.uniform(-.5, .5, (period, 3)).astype(np.float32)
    A = P[np.arange(n_rows) % period][None]
    B = r.uniform(-.5, .5, (1, 500, 3)).astype(np.float32)
    return A, B


def _descending_rows(seed=43):
    """32 row workgroups; target 0 (the origin) has one near row per workgroup at a squared
    distance that falls by 0.15% per workgroup, the other rows lie on a sphere of radius 2.  The
    column merge keeps every near row on its list as it arrives and must drop the early ones once
    they leave the threshold of the falling minimum."""
    r = np.random.default_rng(seed)
    u = r.normal(size=(32 * WG_ROWS, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    A = 2.0 * u
    for w in range(32):
        A[WG_ROWS * w + 5] = np.sqrt(0.1 * (1 - 0.0015 * w)) * u[WG_ROWS * w + 5]
    B = r.uniform(-.5, .5, (1, 100, 3))
    B[0, 0] = 0.0
    return A[None].astype(np.float32), B.astype(np.float32)


COLUMN_MERGE_CASES = {
    "ties-32-workgroups": lambda: _periodic_rows(32 * WG_ROWS),   # list overflows: heavy
    "ties-14-workgroups": lambda: _periodic_rows(14 * WG_ROWS),   # 14 candidates > 12: heavy
    "ties-12-workgroups": lambda: _periodic_rows(12 * WG_ROWS),   # 12 candidates, full rescans
    "descending-minimum": _descending_rows,                       # stale list entries dropped
}


@pytest.mark.parametrize("case", list(COLUMN_MERGE_CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_column_merge_ties_and_list_overflow(case, precision):
    """Targets whose nearest rows tie (or nearly tie) across many row workgroups: the column
    direction must still give the exact argmin with the smallest-index rule, whether the target
    stays light, exceeds the candidate limit or overflows the merge's list."""
    p = gpu()
    say(f"[chamfer] column merge {case} precision={precision}")
    A, B = COLUMN_MERGE_CASES[case]()
    g, o = _chamfer_both(p, A, B, precision=precision)
    _check_chamfer(g, o)
    if case.startswith("ties"):
        assert np.all(g["idx_b"] < 37)


@pytest.mark.parametrize("scale", [1e-12, 1e-6, 1e6, 1e12])
@pytest.mark.parametrize("precision", [0, 1])
def test_coordinate_scales(scale, precision):
    """The screen's certificate scales with the points' norms and its column partials are coded
    over 32 binades placed by each frame's largest norm: clouds at very small and very large
    scales, next to a frame at unit scale and one at the square root of the scale in the same
    call, give the exhaustive search's indices and distances in both directions."""
    p = gpu()
    say(f"[chamfer] scale {scale:g} precision={precision}")
    r = np.random.default_rng(71)
    A = r.uniform(-.5, .5, (3, 5000, 3))
    B = r.uniform(-.5, .5, (3, 4100, 3))
    B[:, :50] = A[:, :50] + r.normal(scale=1e-4, size=(3, 50, 3))  # near pairs
    for t, f in enumerate((scale, 1.0, np.sqrt(scale))):
        A[t] *= f
        B[t] *= f
    A, B = A.astype(np.float32), B.astype(np.float32)
    g, o = _chamfer_both(p, A, B, precision=precision)
    _check_chamfer(g, o)


def test_chamfer_backward_ignores_out_of_range_neighbours():
    """A neighbour index outside [0, N) contributes nothing to the Chamfer gradient (the
    library's rule for indices it did not produce; the sort keeps such entries apart from the
    last valid index).  Expected: the oracle's gradient for the valid indices, less the terms of
    the entries made invalid, in double."""
    p = gpu()
    say("[chamfer] backward with out-of-range neighbour indices")
    r = np.random.default_rng(81)
    T, Na, Nb = 2, 3000, 2500
    A = r.uniform(-.5, .5, (T, Na, 3)).astype(np.float32)
    B = r.uniform(-.5, .5, (T, Nb, 3)).astype(np.float32)
    o = oracle.chamfer(A, B)
    ia, ib = o["idx_a"].copy(), o["idx_b"].copy()
    alpha, beta = 1.0 / Na, 1.0 / Nb
    bad_a = r.random((T, Na)) < 0.05
    bad_b = r.random((T, Nb)) < 0.05
    ib[:, -1] = Na - 1  # the largest valid key, next to the invalid ones
    bad_b[:, -1] = False
    og = oracle.chamfer_grad(A, B, ia, ib, want_b=True)
    ga, gb, gaa, gba = og["ga"].copy(), og["gb"].copy(), og["ga_abs"], og["gb_abs"]
    for t in range(T):
        for i in np.nonzero(bad_a[t])[0]:
            g = 2 * alpha * (A[t, i].astype(np.float64) - B[t, ia[t, i]])
            ga[t, i] -= g
            gb[t, ia[t, i]] += g
        for j in np.nonzero(bad_b[t])[0]:
            g = 2 * beta * (A[t, ib[t, j]].astype(np.float64) - B[t, j])
            ga[t, ib[t, j]] -= g
            gb[t, j] += g
    vals_a = np.array([-1, Nb, 1 << 30], np.int32)
    vals_b = np.array([-1, Na, 1 << 30], np.int32)
    ia[bad_a] = vals_a[r.integers(0, 3, bad_a.sum())]
    ib[bad_b] = vals_b[r.integers(0, 3, bad_b.sum())]
    gA, gB = p.chamfer_bwd(torch.ones(T, dtype=torch.float64, device="cuda"), dev(A), dev(B),
                           dev(ia), dev(ib), want_b=True)
    torch.cuda.synchronize()
    assert_grad(host(gA), ga, gaa, 1e-5, "grad_a")
    assert_grad(host(gB), gb, gba, 1e-5, "grad_b")


def _few_heavy(n, seed):
    """n x n points with a few queries the screen cannot settle in either direction: one row
    point repeated every 256 rows, so every row workgroup of either screen holds it (and the
    targets near it tie across all of them),
    and one target point repeated in 16 different slot groups (so the rows near it have more
    candidate groups than the screen keeps)."""
    r = np.random.default_rng(seed)
    A = r.uniform(-.5, .5, (1, n, 3)).astype(np.float32)
    B = r.uniform(-.5, .5, (1, n, 3)).astype(np.float32)
    X = np.array([0.11, -0.23, 0.05], np.float32)
    Y = np.array([-0.31, 0.17, -0.12], np.float32)
    A[0, 7::256] = X
    B[0, 5:5 + 2048 * 16:2048][: (n - 5 + 2047) // 2048] = Y
    B[0, 10:15] = X + r.normal(scale=1e-3, size=(5, 3)).astype(np.float32)
    A[0, 10:15] = Y + r.normal(scale=1e-3, size=(5, 3)).astype(np.float32)
    return A, B


@pytest.mark.parametrize("n", [6000, 20000])
def test_short_heavy_lists(n):
    """A handful of heavy rows and columns per frame go to the one-wave-per-query search (with
    target slices at 20,000 points, without at 6,000): exact against the oracle, and bitwise equal
    to the exhaustive fp32 path."""
    p = gpu()
    say(f"[chamfer] short heavy lists n={n}")
    A, B = _few_heavy(n, 51)
    ctx = p.Context(0)
    g = p.chamfer_fwd(dev(A), dev(B), precision=1, ctx=ctx)
    ctx.sync()
    st = ctx.stats()
    say(f"[chamfer] {st}")
    assert 0 < st["fallbacks"] <= 64
    ctx.close()
    g = {k: host(v) for k, v in g.items()}
    o = oracle.chamfer(A, B, 0, None)
    _check_chamfer(g, o)


def test_non_finite_points_follow_the_exhaustive_path():
    """Rows or targets at NaN or at a distance whose square overflows are heavy for the screen:
    the bf16 path returns exactly what the exhaustive fp32 path returns (indices and distances,
    bit for bit), whichever list search handles them."""
    p = gpu()
    say("[chamfer] non-finite points")
    r = np.random.default_rng(61)
    for n, bad in ((3000, 3), (20000, 3), (20000, 300)):
        A = r.uniform(-.5, .5, (1, n, 3)).astype(np.float32)
        B = r.uniform(-.5, .5, (1, n, 3)).astype(np.float32)
        rows = r.choice(n, bad, replace=False)
        cols = r.choice(n, bad, replace=False)
        A[0, rows[0::2]] = np.nan
        A[0, rows[1::2], 0] = 3e30
        B[0, cols[0::2], 1] = np.nan
        B[0, cols[1::2]] = -2e30
        g0 = {k: host(v) for k, v in p.chamfer_fwd(dev(A), dev(B), precision=0).items()}
        g1 = {k: host(v) for k, v in p.chamfer_fwd(dev(A), dev(B), precision=1).items()}
        torch.cuda.synchronize()
        for k in ("idx_a", "idx_b", "dist_a", "dist_b"):
            assert np.array_equal(g0[k].view(np.uint32), g1[k].view(np.uint32)), (n, bad, k)
        for k in ("idx_a", "idx_b"):
            assert g1[k].min() >= 0 and g1[k].max() < n


def _many_frames(seed, T, Na, Nb, bad=False):
    """T frames with exact ties (duplicated targets and rows) and, with `bad`, rows and targets at
    NaN or at distances whose square overflows in a few frames."""
    r = np.random.default_rng(seed)
    A = r.uniform(-.5, .5, (T, Na, 3)).astype(np.float32)
    B = r.uniform(-.5, .5, (T, Nb, 3)).astype(np.float32)
    B[:, Nb // 2: Nb // 2 + 40] = B[:, :40]          # duplicated targets: row ties
    A[:, Na // 3: Na // 3 + 40] = A[:, 5:45]         # duplicated rows: column ties
    if bad:
        for t in r.choice(T, 8, replace=False):
            A[t, r.choice(Na, 3, replace=False)] = np.nan
            A[t, r.choice(Na, 2, replace=False), 1] = 4e30
            B[t, r.choice(Nb, 3, replace=False), 2] = np.nan
            B[t, r.choice(Nb, 2, replace=False)] = -3e30
        A[T - 1] = np.nan                            # a frame of NaN rows only
        B[T - 2, :, 0] = 5e30                        # a frame whose targets are all overflowing
    return A, B


@pytest.mark.parametrize("shape", [(300, 1000, 777), (260, 2300, 5000), (1100, 2048, 300)])
def test_one_pass_both_directions(shape):
    """Many frames (the fp32 path then searches both directions in one pass over the pairs): equal
    to the oracle element by element, and, with NaN and overflowing points added, bit for bit equal
    to the two single-direction searches that smaller calls of the same frames use."""
    p = gpu()
    T, Na, Nb = shape
    say(f"[chamfer] one pass both directions T={T} Na={Na} Nb={Nb}")
    A, B = _many_frames(7 + T, T, Na, Nb)
    g, o = _chamfer_both(p, A, B, precision=0)
    _check_chamfer(g, o)
    A, B = _many_frames(8 + T, T, Na, Nb, bad=True)
    whole = {k: host(v) for k, v in p.chamfer_fwd(dev(A), dev(B), precision=0).items()}
    torch.cuda.synchronize()
    for t in sorted({0, T - 2, T - 1} | set(range(1, T, max(1, T // 12)))):
        part = {k: host(v) for k, v in
                p.chamfer_fwd(dev(A[t:t + 1]), dev(B[t:t + 1]), precision=0).items()}
        for k in ("idx_a", "idx_b", "dist_a", "dist_b"):
            assert np.array_equal(whole[k][t].view(np.uint32), part[k][0].view(np.uint32)), (t, k)


def test_maximum_frame_count():
    """T = 65,535 frames (the largest the ABI takes) of a single triangle: sampling, both Chamfer
    directions in both precisions, and the backward to vertices, element by element against the
    oracle (grids of 65,535 frames in every kernel)."""
    p = gpu()
    say("[limits] 65535 frames")
    T, N, Nb = 65535, 5, 3
    r = np.random.default_rng(81)
    verts = r.uniform(-.5, .5, (T, 3, 3)).astype(np.float32)
    faces = np.array([[0, 1, 2]], np.int32)
    obs = r.uniform(-.5, .5, (T, Nb, 3)).astype(np.float32)
    gp, gf, gb = p.sample_surface(dev(verts), dev(faces), N, seed=99)
    op, of, ob = oracle.sample_surface(verts, faces, N, seed=99)
    assert np.array_equal(host(gf), of)
    assert np.array_equal(host(gp).view(np.uint32), op.view(np.uint32))
    o = oracle.chamfer(op, obs)
    og = oracle.chamfer_grad(op, obs, o["idx_a"], o["idx_b"])
    ogv, ogva = oracle.sample_grad(og["ga"], faces, of, ob, 3, og["ga_abs"])
    for precision in (0, 1):
        f = p.chamfer_fwd(gp, dev(obs), precision=precision)
        ga, _ = p.chamfer_bwd(torch.ones(T, dtype=torch.float64, device="cuda"), gp, dev(obs),
                              f["idx_a"], f["idx_b"])
        gv = p.sample_surface_bwd(ga, dev(faces), gf, gb, 3)
        torch.cuda.synchronize()
        _check_chamfer({k: host(v) for k, v in f.items()}, o)
        assert_grad(host(gv), ogv, ogva, what="grad_verts")


@pytest.mark.parametrize("shape", [((1 << 24), 7), (7, (1 << 24))])
@pytest.mark.parametrize("precision", [0, 1])
def test_maximum_point_count(shape, precision):
    """2^24 points (the largest count the ABI takes) against a handful on the other side, both
    ways round, both precisions: indices exact and float distances bit for bit in both
    directions."""
    p = gpu()
    Na, Nb = shape
    say(f"[limits] {Na} x {Nb} precision={precision}")
    r = np.random.default_rng(83)
    A = r.uniform(-.5, .5, (1, Na, 3)).astype(np.float32)
    B = r.uniform(-.5, .5, (1, Nb, 3)).astype(np.float32)
    g, o = _chamfer_both(p, A, B, precision=precision)
    _check_chamfer(g, o)


@pytest.mark.parametrize("reduction", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_loss_reductions_and_weights(reduction, precision):
    p = gpu()
    r = np.random.default_rng(31)
    A = r.uniform(-.5, .5, (3, 500, 3)).astype(np.float32)
    B = r.uniform(-.5, .5, (3, 700, 3)).astype(np.float32)
    w = np.array([0.5, 0.0, 2.0], np.float32)
    g, o = _chamfer_both(p, A, B, reduction=reduction, frame_w=w, precision=precision)
    _check_chamfer(g, o)


@pytest.mark.parametrize("case", ["cfg1", "cfg2-3frames", "ragged-1000x4097", "slices-2x20000"])
@pytest.mark.parametrize("precision", [0, 1])
def test_unidirectional_fast_path(case, precision):
    """Eq. 2 with the b outputs omitted searches only a -> b (the bf16 path runs its row-only
    screen): idx_a / dist_a equal the oracle bit for bit, the loss matches, and both equal the
    bidirectional call's; the gradient to a needs no idx_b."""
    p = gpu()
    A, B = CHAMFER_CASES[case]()
    say(f"[chamfer] unidirectional {case} precision={precision}")
    w = np.linspace(0.5, 1.5, A.shape[0]).astype(np.float32)
    g1 = p.chamfer_fwd(dev(A), dev(B), precision=precision, reduction=1, frame_w=dev(w),
                       b_side=False)
    g2 = p.chamfer_fwd(dev(A), dev(B), precision=precision, reduction=1, frame_w=dev(w))
    gl = torch.full((A.shape[0],), 2.0, dtype=torch.float64, device="cuda")
    ga1, gb1 = p.chamfer_bwd(gl, dev(A), dev(B), g1["idx_a"], None, reduction=1, frame_w=dev(w),
                             want_b=True)
    ga2, gb2 = p.chamfer_bwd(gl, dev(A), dev(B), g2["idx_a"], g2["idx_b"], reduction=1,
                             frame_w=dev(w), want_b=True)
    torch.cuda.synchronize()
    assert g1["idx_b"] is None and g1["dist_b"] is None
    o = oracle.chamfer(A, B, 1, w)
    assert np.array_equal(host(g1["idx_a"]), o["idx_a"])
    assert np.array_equal(host(g1["dist_a"]).view(np.uint32), o["d32a"].view(np.uint32))
    assert_rel(host(g1["loss"]), o["loss"], 1e-5, "loss")
    assert np.array_equal(host(g1["loss"]).view(np.uint64), host(g2["loss"]).view(np.uint64))
    assert torch.equal(ga1, ga2) and torch.equal(gb1, gb2)
    og = oracle.chamfer_grad(A, B, o["idx_a"], o["idx_b"], 1, w, np.full(A.shape[0], 2.0),
                             want_b=True)
    assert_grad(host(ga1), og["ga"], og["ga_abs"], what="grad a")
    assert_grad(host(gb1), og["gb"], og["gb_abs"], what="grad b")


def test_unidirectional_argument_checks():
    p = gpu()
    A = dev(np.zeros((1, 8, 3), np.float32))
    with pytest.raises(p.DCError):  # Eq. 1 needs the b side
        p.chamfer_fwd(A, A, reduction=0, b_side=False)
    ia = torch.zeros((1, 8), dtype=torch.int32, device="cuda")
    gl = torch.ones(1, dtype=torch.float64, device="cuda")
    with pytest.raises(p.DCError):
        p.chamfer_bwd(gl, A, A, ia, None, reduction=0)


def test_screen_candidates_are_few():
    """The bf16 screen's certificate must leave only a handful of candidate groups per query and
    rarely fall back to an exhaustive search (otherwise the screen would be pointless)."""
    p = gpu()
    say("[screen] candidate statistics, 100x100 grid, 2 frames of 65536 x 65536")
    w = gen.workload(4, T=2)
    ctx = p.Context(0)
    pts, _, _ = p.sample_surface(dev(w["verts"]), dev(w["faces"]), w["Na"], seed=w["seed"],
                                 ctx=ctx)
    p.chamfer_fwd(pts, dev(w["observed"]), precision=1, ctx=ctx)
    ctx.sync()
    st = ctx.stats()
    say(f"[screen] {st}")
    q = st["queries"]
    assert q == 2 * 2 * 65536
    assert st["candidates"] / q < 8
    assert st["fallbacks"] / q < 0.05
    ctx.close()


@pytest.mark.parametrize("cfg,T", [(1, None), (3, None), (2, 2)])
@pytest.mark.parametrize("reduction", [0, 1])
def test_backward_parity(cfg, T, reduction):
    """Chamfer backward and sampling backward against the oracle's double gradients."""
    p = gpu()
    say(f"[backward] cfg{cfg} reduction={reduction}")
    w = gen.workload(cfg, T=T)
    verts, faces, obs, words = w["verts"], w["faces"], w["observed"], w["words"]
    Tn = verts.shape[0]
    fw = np.linspace(0.5, 1.5, Tn).astype(np.float32)
    gl = np.linspace(1.0, -0.5, Tn)
    pts, fi, ba = oracle.sample_surface(verts, faces, w["Na"], words=words)
    och = oracle.chamfer(pts, obs, reduction, fw)
    og = oracle.chamfer_grad(pts, obs, och["idx_a"], och["idx_b"], reduction, fw, gl,
                             want_b=True)
    ogv, ogva = oracle.sample_grad(og["ga"], faces, fi, ba, w["V"], og["ga_abs"])
    # GPU pipeline on the same inputs
    gpts, gfi, gba = p.sample_surface(dev(verts), dev(faces), w["Na"],
                                      uniforms=dev(words.view(np.int32)))
    fwd = p.chamfer_fwd(gpts, dev(obs), reduction=reduction, frame_w=dev(fw))
    ga, gb = p.chamfer_bwd(dev(gl), gpts, dev(obs), fwd["idx_a"], fwd["idx_b"],
                           reduction=reduction, frame_w=dev(fw), want_b=True)
    gv = p.sample_surface_bwd(ga, dev(faces), gfi, gba, w["V"])
    torch.cuda.synchronize()
    assert np.array_equal(host(fwd["idx_a"]), och["idx_a"])
    assert_grad(host(ga), og["ga"], og["ga_abs"], what="grad_a")
    assert_grad(host(gb), og["gb"], og["gb_abs"], what="grad_b")
    assert_grad(host(gv), ogv, ogva, what="grad_verts")


def _segment_cases():
    """Shapes at the edges of the backward's segments: one row (every target's neighbour is
    row 0: one segment holds every key), one target, all targets at one point (one segment of
    the whole frame, the other keys empty at both ends), and a ragged size."""
    r = np.random.default_rng(91)
    u = lambda *s: r.uniform(-.5, .5, s).astype(np.float32)  # noqa: E731
    same = np.repeat(u(2, 1, 3), 700, axis=1)
    # the neighbour sorts either side of the one-workgroup sort's limit of 4,096 keys: idx_b
    # (4,096 keys) in one workgroup, idx_a (4,097) in the block passes
    cut = (u(2, 4097, 3), u(2, 4096, 3))
    return {"one-row": (u(2, 1, 3), u(2, 7, 3)), "one-target": (u(1, 300, 3), u(1, 1, 3)),
            "one-point-targets": (u(2, 900, 3), same), "ragged": (u(3, 1001, 3), u(3, 777, 3)),
            "sort-cutover": cut}


@pytest.mark.parametrize("case", ["one-row", "one-target", "one-point-targets", "ragged",
                                  "sort-cutover"])
@pytest.mark.parametrize("precision", [0, 1])
def test_backward_segment_edges(case, precision):
    """The Chamfer backward at the edges of its neighbour segments, in both directions, against
    the oracle's double gradient (indices from the forward equal the oracle's)."""
    p = gpu()
    say(f"[backward] segments {case} precision={precision}")
    A, B = _segment_cases()[case]
    T = A.shape[0]
    gl = np.linspace(1.0, 0.25, T)
    o = oracle.chamfer(A, B)
    og = oracle.chamfer_grad(A, B, o["idx_a"], o["idx_b"], 0, None, gl, want_b=True)
    f = p.chamfer_fwd(dev(A), dev(B), precision=precision)
    ga, gb = p.chamfer_bwd(dev(gl), dev(A), dev(B), f["idx_a"], f["idx_b"], want_b=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(f["idx_a"]), o["idx_a"])
    assert np.array_equal(host(f["idx_b"]), o["idx_b"])
    assert_grad(host(ga), og["ga"], og["ga_abs"], what="grad_a")
    assert_grad(host(gb), og["gb"], og["gb_abs"], what="grad_b")


@pytest.mark.parametrize("N", [4096, 4097])
def test_sampling_backward_at_sort_cutover(N):
    """Eq. 4 with the points-by-face sort (two digit passes over 1,682 faces) on either side of
    the one-workgroup sort's limit: 4,096 points per frame in one workgroup, 4,097 in the block
    passes; vertex gradients against the oracle's double sums."""
    p = gpu()
    say(f"[backward] sampling sort cutover N={N}")
    verts, faces = gen.trajectory(30, 2, 4)
    T, V = verts.shape[:2]
    r = np.random.default_rng(N)
    words = r.integers(0, 2**32, size=(T, N, 4), dtype=np.uint64).astype(np.uint32)
    gp = r.standard_normal((T, N, 3)).astype(np.float32)
    _, fi, ba = p.sample_surface(dev(verts), dev(faces), N, uniforms=dev(words.view(np.int32)))
    gv = p.sample_surface_bwd(dev(gp), dev(faces), fi, ba, V)
    torch.cuda.synchronize()
    ogv, ogva = oracle.sample_grad(gp, faces, host(fi), host(ba), V, np.abs(gp))
    assert_grad(host(gv), ogv, ogva, what="grad_verts")


def test_determinism():
    p = gpu()
    w = gen.workload(3)
    verts, faces, obs = dev(w["verts"]), dev(w["faces"]), dev(w["observed"])
    outs = []
    for _ in range(2):
        pts, fi, ba = p.sample_surface(verts, faces, w["Na"], seed=5)
        f = p.chamfer_fwd(pts, obs)
        ga, gb = p.chamfer_bwd(torch.ones(w["T"], dtype=torch.float64, device="cuda"), pts, obs,
                               f["idx_a"], f["idx_b"], want_b=True)
        gv = p.sample_surface_bwd(ga, faces, fi, ba, w["V"])
        outs.append([host(x).copy() for x in (pts, f["idx_a"], f["idx_b"], f["loss"], ga, gb, gv)])
    for x, y in zip(*outs):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


def test_calls_on_two_streams():
    """Direct calls of one context issued back to back on two streams share its scratch memory:
    the second waits for the first on the device, and both return exactly the results of calls
    made one after the other on one stream."""
    p = gpu()
    say("[streams] two streams, one context")
    r = np.random.default_rng(71)
    A1 = dev(r.uniform(-.5, .5, (24, 32768, 3)).astype(np.float32))
    B1 = dev(r.uniform(-.5, .5, (24, 32768, 3)).astype(np.float32))
    A2 = dev(r.uniform(-.5, .5, (3, 5000, 3)).astype(np.float32))
    B2 = dev(r.uniform(-.5, .5, (3, 7000, 3)).astype(np.float32))
    ctx = p.Context(0)
    ref1 = {k: host(v).copy() for k, v in p.chamfer_fwd(A1, B1, precision=1, ctx=ctx).items()}
    ref2 = {k: host(v).copy() for k, v in p.chamfer_fwd(A2, B2, precision=1, ctx=ctx).items()}
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        g1 = p.chamfer_fwd(A1, B1, precision=1, ctx=ctx)
    with torch.cuda.stream(s2):
        g2 = p.chamfer_fwd(A2, B2, precision=1, ctx=ctx)
    torch.cuda.synchronize()
    for ref, g in ((ref1, g1), (ref2, g2)):
        for k, v in ref.items():
            assert np.array_equal(host(g[k]).view(np.uint8), v.view(np.uint8)), k
    ctx.close()


def _frame_oracle(verts, faces, obs, seed, t, Na, V, reduction):
    """The oracle's whole pipeline on frame t alone: Philox words of (seed, t), sampling, the
    exhaustive nearest neighbours both ways, the loss, and the double gradients to the points,
    to the observed cloud and (through Eq. 4) to the vertices."""
    op, ofi, oba = oracle.sample_surface(verts[t:t + 1], faces, Na,
                                         words=_words_frame(seed, t, Na))
    och = oracle.chamfer(op, obs[t:t + 1], reduction)
    og = oracle.chamfer_grad(op, obs[t:t + 1], och["idx_a"], och["idx_b"], reduction,
                             want_b=True)
    ogv, ogva = oracle.sample_grad(og["ga"], faces, ofi, oba, V, og["ga_abs"])
    return dict(points=op[0], face_idx=ofi[0], bary=oba[0], ch=och, g=og, gv=ogv[0],
                gva=ogva[0])


def _check_whole_frame(o, t, g, both=True):
    """Element-wise comparison of frame t of the GPU outputs `g` (host arrays of the whole
    trajectory) with the oracle's frame `o`."""
    och = o["ch"]
    assert np.array_equal(g["face_idx"][t], o["face_idx"])
    assert np.array_equal(g["points"][t].view(np.uint32), o["points"].view(np.uint32))
    assert np.array_equal(g["bary"][t].view(np.uint32), o["bary"].view(np.uint32))
    assert np.array_equal(g["idx_a"][t], och["idx_a"][0])
    assert np.array_equal(g["dist_a"][t].view(np.uint32), och["d32a"][0].view(np.uint32))
    nz = och["d64a"][0] > 0
    assert_rel(g["dist_a"][t][nz], och["d64a"][0][nz], 1e-5, "dist_a vs double")
    if both:
        assert np.array_equal(g["idx_b"][t], och["idx_b"][0])
        assert np.array_equal(g["dist_b"][t].view(np.uint32), och["d32b"][0].view(np.uint32))
        nz = och["d64b"][0] > 0
        assert_rel(g["dist_b"][t][nz], och["d64b"][0][nz], 1e-5, "dist_b vs double")
        assert_grad(g["grad_b"][t], o["g"]["gb"][0], o["g"]["gb_abs"][0], what="grad_b")
    assert_rel(g["loss"][t:t + 1], och["loss"], 1e-5, "loss")
    assert_grad(g["grad_a"][t], o["g"]["ga"][0], o["g"]["ga_abs"][0], what="grad_a")
    assert_grad(g["grad_verts"][t], o["gv"], o["gva"], what="grad_verts")


def _gpu_pipeline(p, w, precision, reduction, both=True):
    """The whole path on the GPU for every frame of workload `w` (sampler keyed by its seed, as
    the benchmark runs it); host copies of every output."""
    verts, faces, obs = dev(w["verts"]), dev(w["faces"]), dev(w["observed"])
    T = w["T"]
    pts, fi, ba = p.sample_surface(verts, faces, w["Na"], seed=w["seed"])
    f = p.chamfer_fwd(pts, obs, precision=precision, reduction=reduction, b_side=both)
    ga, gb = p.chamfer_bwd(torch.ones(T, dtype=torch.float64, device="cuda"), pts, obs,
                           f["idx_a"], f["idx_b"], reduction=reduction, want_b=both)
    gv = p.sample_surface_bwd(ga, faces, fi, ba, w["V"])
    torch.cuda.synchronize()
    out = dict(points=pts, face_idx=fi, bary=ba, grad_a=ga, grad_b=gb, grad_verts=gv, **f)
    return {k: (None if v is None else host(v)) for k, v in out.items()}


@pytest.mark.parametrize("reduction", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_trajectory_workload_full(precision, reduction):
    """The 40-frame, 50x50-grid, 8,192 x 8,192 trajectory workload at its stated size, every
    frame element by element: faces, points and weights bit for bit, neighbour indices exact in
    both directions, float distances bit for bit (and within 1e-5 of the double twin), losses
    within 1e-5, gradients to the points, the observed cloud and the vertices within 1e-5 of the
    sum of absolute contributions (Sec. III-A Eq. 1-2, Sec. III-B Eq. 3-4)."""
    p = gpu()
    say(f"[trajectory] 40 frames 8192x8192 precision={precision} reduction={reduction}")
    w = gen.workload(2)
    assert w["T"] == 40 and w["Na"] == 8192 and w["Nb"] == 8192
    g = _gpu_pipeline(p, w, precision, reduction)
    verts, faces, obs, T, Na = w["verts"], w["faces"], w["observed"], w["T"], w["Na"]
    op, ofi, oba = oracle.sample_surface(verts, faces, Na, seed=w["seed"])
    assert np.array_equal(g["face_idx"], ofi)
    assert np.array_equal(g["points"].view(np.uint32), op.view(np.uint32))
    assert np.array_equal(g["bary"].view(np.uint32), oba.view(np.uint32))
    och = oracle.chamfer(op, obs, reduction)
    _check_chamfer(g, och)
    og = oracle.chamfer_grad(op, obs, och["idx_a"], och["idx_b"], reduction, want_b=True)
    assert_grad(g["grad_a"], og["ga"], og["ga_abs"], what="grad_a")
    assert_grad(g["grad_b"], og["gb"], og["gb_abs"], what="grad_b")
    ogv, ogva = oracle.sample_grad(og["ga"], faces, ofi, oba, w["V"], og["ga_abs"])
    assert_grad(g["grad_verts"], ogv, ogva, what="grad_verts")


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_sampled(precision):
    """The 100-frame, 65,536 x 65,536 workload in the benchmark's launch configuration: one whole
    frame (drawn at random) element by element against the oracle (faces, points, indices and
    distances in both directions, loss, gradients to points, observed cloud and vertices); on
    three more frames sampled points bit for bit and the neighbours of sampled queries (the oracle
    searches the full frame for each); and properties of the whole gradient that hold at any
    size."""
    p = gpu()
    say(f"[full-size] precision={precision}")
    w = gen.workload(4)
    verts, faces, obs = w["verts"], w["faces"], w["observed"]
    T, Na, Nb = w["T"], w["Na"], w["Nb"]
    g = _gpu_pipeline(p, w, precision, 0)
    r = np.random.default_rng(44 + precision)
    t_whole = int(r.integers(T))
    say(f"[full-size] whole frame {t_whole}")
    _check_whole_frame(_frame_oracle(verts, faces, obs, w["seed"], t_whole, Na, w["V"], 0),
                       t_whole, g)
    hp, hfi, ia, ib = g["points"], g["face_idx"], g["idx_a"], g["idx_b"]
    frames = sorted(r.choice(T, 3, replace=False))
    for t in frames:
        op, ofi, _ = oracle.sample_surface(verts[t:t + 1], faces, Na,
                                           words=_words_frame(w["seed"], t, Na))
        assert np.array_equal(hfi[t], ofi[0])
        assert np.array_equal(hp[t].view(np.uint32), op[0].view(np.uint32))
        qa = r.choice(Na, 48, replace=False)
        oi, od, _ = oracle.nearest(op[0][qa], obs[t])
        assert np.array_equal(ia[t][qa], oi)
        qb = r.choice(Nb, 48, replace=False)
        oi, od, _ = oracle.nearest(obs[t][qb], op[0])
        assert np.array_equal(ib[t][qb], oi)
    # whole-gradient properties: translation invariance makes every frame's a- and b-gradients
    # sum to zero; Eq. 4 weights sum to one, so vertex gradients sum to the point gradients
    ga, gb, gv = g["grad_a"], g["grad_b"], g["grad_verts"]
    sa = ga.astype(np.float64).sum(1)
    sb = gb.astype(np.float64).sum(1)
    scale = np.abs(ga).astype(np.float64).sum(1) + 1e-30
    assert np.all(np.abs(sa + sb) <= 1e-4 * scale)
    sv = gv.astype(np.float64).sum(1)
    assert np.all(np.abs(sv - sa) <= 1e-4 * scale)


def test_full_size_unidirectional_sampled():
    """Eq. 2 on the 100-frame, 65,536 x 65,536 workload in the benchmark's launch configuration
    (the bf16 row-only screen, no b outputs): one whole frame element by element against the
    oracle (indices and distances bit for bit, loss, gradients to the points and vertices);
    sampled rows of three more frames bit for bit; every frame's loss equals the sum of its row
    distances."""
    p = gpu()
    say("[full-size] unidirectional bf16")
    w = gen.workload(4)
    verts, faces, obs = w["verts"], w["faces"], w["observed"]
    T, Na = w["T"], w["Na"]
    g = _gpu_pipeline(p, w, 1, 1, both=False)
    assert g["idx_b"] is None
    r = np.random.default_rng(45)
    t_whole = int(r.integers(T))
    say(f"[full-size] whole frame {t_whole}")
    _check_whole_frame(_frame_oracle(verts, faces, obs, w["seed"], t_whole, Na, w["V"], 1),
                       t_whole, g, both=False)
    hp, ia, da = g["points"], g["idx_a"], g["dist_a"]
    for t in sorted(r.choice(T, 3, replace=False)):
        qa = r.choice(Na, 48, replace=False)
        oi, od, _ = oracle.nearest(hp[t][qa], obs[t])
        assert np.array_equal(ia[t][qa], oi)
        assert np.array_equal(da[t][qa].view(np.uint32), od.view(np.uint32))
    # Eq. 2: the frame loss is the plain sum of the frame's squared distances
    assert_rel(g["loss"], da.astype(np.float64).sum(1), 1e-5, "loss")


def test_face_choice_at_the_top_of_the_range():
    """Face choice with the largest face word (all 53 bits set, r = 1 - 2^-53) on a mesh whose
    last faces are outside the subset: r S stays below S, so the first face whose running sum
    exceeds it is the last face of nonzero area, never one of the trailing excluded faces; the
    same with the smallest word (r = 0: the first face of nonzero area).  Points, weights and
    faces bit for bit against the oracle."""
    p = gpu()
    say("[sample] top and bottom of the face-word range, trailing excluded faces")
    verts, faces = gen.trajectory(12, 3, 4)
    F = len(faces)
    N = 64
    words = np.zeros((3, N, 4), np.uint32)
    words[:, : N // 2, 0] = 0xFFFFFFFF
    words[:, : N // 2, 1] = 0xFFFFFFFF
    words[:, :, 2] = np.arange(N, dtype=np.uint32) << 20
    words[:, :, 3] = np.arange(N, dtype=np.uint32)[::-1] << 21
    mask = np.ones((3, F), np.uint8)
    mask[0, F - 5:] = 0     # five trailing excluded faces
    mask[1, F - 1:] = 0     # one
    mask[2, :7] = 0         # leading excluded faces: r = 0 must skip them
    m = torch.from_numpy(mask).to("cuda")
    g = p.sample_surface(dev(verts), dev(faces), N, uniforms=dev(words.view(np.int32)),
                         face_mask=m)
    gp, gf, gb = (host(x) for x in g)
    o = oracle.sample_surface(verts, faces, N, words=words, face_mask=mask)
    assert np.array_equal(gf, o[1])
    assert np.array_equal(gp.view(np.uint32), o[0].view(np.uint32))
    assert np.array_equal(gb.view(np.uint32), o[2].view(np.uint32))
    last = [int(np.nonzero(mask[t])[0].max()) for t in range(3)]
    first = [int(np.nonzero(mask[t])[0].min()) for t in range(3)]
    for t in range(3):
        assert np.all(gf[t, : N // 2] == last[t])
        assert np.all(gf[t, N // 2:] == first[t])


def _words_frame(seed, t, N):
    """Philox words of one frame t (the generator is keyed by frame, so a frame can be drawn
    alone)."""
    full = np.zeros((1, N, 4), np.uint32)
    c = oracle.words_from_seed(seed, t + 1, N)
    full[0] = c[t]
    return full
