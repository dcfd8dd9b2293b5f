"""Pins of the CPU oracle against things other than itself: hand-derived examples, closed forms,
invariants, statistics, an independent library generator, and exact brute force (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import gen

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")))


# ----------------------------------------------------------------- random words
def _numpy_philox(ctr, key):
    c = sum(int(x) << (64 * k) for k, x in enumerate(ctr))
    k = int(key[0]) | (int(key[1]) << 64)
    # numpy's generator increments its 256-bit counter before each block
    return np.random.Philox(counter=(c - 1) % (1 << 256), key=k).random_raw(4)


@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((5, 7, 0, 0), (123, 0)),
                                     ((2**64 - 1, 3, 9, 11), (2**63 + 5, 77)),
                                     ((65535, 99, 0, 0), (1004, 0))])
def test_philox_matches_numpy(ctr, key):
    got = oracle.philox4x64_10(np.array(ctr, np.uint64), np.array(key, np.uint64))
    assert np.array_equal(got, _numpy_philox(ctr, key))


def test_words_from_seed_layout():
    w = oracle.words_from_seed(77, 2, 3)
    for t in range(2):
        for i in range(3):
            x = _numpy_philox((i, t, 0, 0), (77, 0))
            exp = [int(x[0]) & 0xFFFFFFFF, int(x[0]) >> 32, int(x[1]) >> 32, int(x[2]) >> 32]
            assert list(map(int, w[t, i])) == exp


# ----------------------------------------------------------------- sampling
def test_sampler_hand_example():
    g = GOLD["sampler_unit_triangle"]
    x, b = oracle.barycentric(g["p1"], g["p2"], g["p3"], g["word_r1"], g["word_r2"])
    assert list(map(float, b)) == g["bary"]
    assert list(map(float, x)) == g["point"]


def test_face_choice_boundary():
    g = GOLD["face_choice_boundary"]
    verts = np.array([p for tri in g["triangles"] for p in tri], np.float32)
    faces = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    A = oracle.face_areas(verts, faces)
    assert list(A) == g["areas"]
    C, rc = oracle.area_cdf(A)
    assert rc == 0 and list(C) == g["cdf"]
    assert oracle.pick_face(A, C, *g["word_at_boundary"]) == g["face_at_boundary"]
    assert oracle.pick_face(A, C, *g["word_below_boundary"]) == g["face_below_boundary"]


def test_zero_area_faces_never_chosen():
    areas = np.array([0.0, 1.0, 0.0, 0.0, 2.0, 0.0])
    C, rc = oracle.area_cdf(areas)
    assert rc == 0
    # r = 0 must skip the leading zero-area face; r just below 1 must not pick the tail
    assert oracle.pick_face(areas, C, 0, 0) == 1
    assert oracle.pick_face(areas, C, 0xFFFFFFFF, 0xFFFFFFFF) == 4
    words = gen.sim_uniform_words(1, 4000, 99)[0]
    got = {oracle.pick_face(areas, C, int(w[0]), int(w[1])) for w in words}
    assert got == {1, 4}


def test_degenerate_total_area():
    _, rc = oracle.area_cdf(np.zeros(5))
    assert rc == -5
    _, rc = oracle.area_cdf(np.array([1.0, np.nan]))
    assert rc == -5
    verts = np.zeros((1, 3, 3), np.float32)  # all corners coincide
    with pytest.raises(oracle.OracleError):
        oracle.sample_surface(verts, np.array([[0, 1, 2]], np.int32), 4, seed=1)


def test_area_closed_forms():
    # right triangle with legs 3 and 4 in an arbitrary plane orientation -> area 6
    v = np.array([[0, 0, 0], [3, 0, 0], [0, 4, 0]], np.float32)
    assert oracle.face_areas(v, np.array([[0, 1, 2]], np.int32))[0] == 6.0
    v2 = v[:, [2, 0, 1]].copy()  # permuted axes: same area
    assert oracle.face_areas(v2, np.array([[0, 1, 2]], np.int32))[0] == 6.0
    # equilateral triangle of side 1: sqrt(3)/4
    eq = np.array([[0, 0, 0], [1, 0, 0], [0.5, math.sqrt(3) / 2, 0]], np.float32)
    a = oracle.face_areas(eq, np.array([[0, 1, 2]], np.int32))[0]
    assert abs(a - math.sqrt(3) / 4) < 1e-7
    # a flat n x n grid over the unit square has total area exactly 1 (every area is a
    # power-of-two multiple for n-1 a power of two)
    xy, faces = gen.grid_mesh(17)
    flat = np.concatenate([xy, np.zeros((xy.shape[0], 1))], 1).astype(np.float32)
    A = oracle.face_areas(flat, faces)
    assert np.all(A == 0.5 / 256) and math.fsum(A) == 1.0
    # scaling every coordinate by 2 scales every area by exactly 4
    verts, faces = gen.trajectory(9, 1, 3)
    A1 = oracle.face_areas(verts[0], faces)
    A2 = oracle.face_areas(verts[0] * 2, faces)
    assert np.array_equal(A2, 4 * A1)


def test_cdf_is_running_sum():
    verts, faces = gen.trajectory(30, 1, 2)
    A = oracle.face_areas(verts[0], faces)
    C, rc = oracle.area_cdf(A)
    assert rc == 0
    assert np.all(np.diff(C) >= 0)
    assert abs(C[-1] - math.fsum(A)) <= len(A) * 2**-53 * C[-1]
    for k in (0, 1, 100, len(A) - 1):
        assert abs(C[k] - math.fsum(A[: k + 1])) <= (k + 1) * 2**-53 * C[k]


def test_sampler_matches_brute_force():
    verts, faces = gen.trajectory(4, 2, 5)
    words = gen.sim_uniform_words(2, 40, 5)
    pts, fi, ba = oracle.sample_surface(verts, faces, 40, words=words)
    for t in range(2):
        areas = [brute.tri_area(*(verts[t][faces[f][c]] for c in range(3)))
                 for f in range(len(faces))]
        assert np.array_equal(np.array(areas), oracle.face_areas(verts[t], faces))
        for i in range(40):
            w = [int(x) for x in words[t, i]]
            f = brute.pick_face(areas, w[0], w[1])
            assert f == fi[t, i]
            x, b = brute.barycentric(*(verts[t][faces[f][c]] for c in range(3)), w[2], w[3])
            assert list(map(float, pts[t, i])) == x
            assert list(map(float, ba[t, i])) == b


def test_masked_sampler_matches_brute_force():
    """Subset sampling (Sec. IV): faces outside the mask take part with area 0.  Checked against
    exact brute force on the masked areas, for a shared [F] mask and a per-frame [T,F] mask that
    leaves runs of consecutive excluded faces."""
    verts, faces = gen.trajectory(5, 2, 5)
    F = len(faces)
    words = gen.sim_uniform_words(2, 60, 6)
    shared = (np.arange(F) % 3 != 1).astype(np.uint8)
    per_frame = np.stack([(np.arange(F) // 4) % 2 == t for t in range(2)]).astype(np.uint8)
    for mask in (shared, per_frame):
        pts, fi, ba, A, C = oracle.sample_surface(verts, faces, 60, words=words, return_cdf=True,
                                                  face_mask=mask)
        for t in range(2):
            m = mask if mask.ndim == 1 else mask[t]
            areas = [brute.tri_area(*(verts[t][faces[f][c]] for c in range(3))) if m[f] else 0.0
                     for f in range(F)]
            assert np.array_equal(np.array(areas), A[t])
            assert not np.any(m[fi[t]] == 0)  # never an excluded face
            for i in range(60):
                w = [int(x) for x in words[t, i]]
                f = brute.pick_face(areas, w[0], w[1])
                assert f == fi[t, i]
                x, b = brute.barycentric(*(verts[t][faces[f][c]] for c in range(3)), w[2], w[3])
                assert list(map(float, pts[t, i])) == x


def test_masked_face_choice_hand_example():
    """Areas (1, 2, 3) with the middle face excluded: the CDF is (1, 1, 4), so r = 1/4 (target
    exactly 1) must skip the excluded face and pick face 2; r just below 1/4 picks face 0."""
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0],      # area 1
                      [0, 0, 1], [2, 0, 1], [0, 2, 1],      # area 2
                      [0, 0, 2], [3, 0, 2], [0, 2, 2]],     # area 3
                     np.float32)
    faces = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]], np.int32)
    # r = (w >> 11) 2^-53 for the 64-bit word w = (hi << 32) | lo
    quarter = (1 << 51) << 11              # r = 2^51 2^-53 = 1/4
    below = ((1 << 51) - 1) << 11          # one 53-bit step below 1/4
    words = np.zeros((1, 2, 4), np.uint32)
    for i, w in enumerate((quarter, below)):
        words[0, i, 0] = w & 0xFFFFFFFF
        words[0, i, 1] = w >> 32
    _, fi, _, A, C = oracle.sample_surface(verts, faces, 2, words=words, return_cdf=True,
                                           face_mask=np.array([1, 0, 1], np.uint8))
    assert list(A[0]) == [1.0, 0.0, 3.0] and list(C[0]) == [1.0, 1.0, 4.0]
    assert list(fi[0]) == [2, 0]


def test_masked_sampler_statistics_and_empty_mask():
    from scipy import stats
    verts, faces = gen.trajectory(8, 1, 7, sag=0.0)
    F = len(faces)
    # upper half of the cloth (y > 0), as in the occlusion heuristic of the fold scenario
    upper = (verts[0][faces][:, :, 1].mean(axis=1) > 0).astype(np.uint8)
    N = 100_000
    _, fi, _ = oracle.sample_surface(verts, faces, N, seed=77, face_mask=upper)
    A = oracle.face_areas(verts[0], faces) * upper
    counts = np.bincount(fi[0], minlength=F)
    assert counts[upper == 0].sum() == 0
    keep = upper == 1
    assert stats.chisquare(counts[keep], A[keep] / A.sum() * N).pvalue > 1e-4
    with pytest.raises(oracle.OracleError):  # nothing left to draw from: zero total area
        oracle.sample_surface(verts, faces, 4, seed=1, face_mask=np.zeros(F, np.uint8))


def test_sqrt_words_exhaustive_sample():
    # every r1 word maps through a correctly rounded float square root; spot-check a spread
    # of the 2^24 levels against the exact-rational rounding
    for k in list(range(0, 2**24, 9973)) + [1, 2, 3, 2**24 - 1, 2**22, 2**23 + 1]:
        r1 = k * 2.0**-24
        assert brute.sqrt32(r1) == float(np.sqrt(np.float32(r1)))


def test_sampler_statistics():
    from scipy import stats
    verts, faces = gen.trajectory(6, 1, 4, sag=0.0)
    N = 200_000
    pts, fi, ba = oracle.sample_surface(verts, faces, N, seed=2024)
    A = oracle.face_areas(verts[0], faces)
    counts = np.bincount(fi[0], minlength=len(faces))
    chi = stats.chisquare(counts, A / A.sum() * N)
    assert chi.pvalue > 1e-4
    # u = 1 - sqrt(r1) has CDF 1 - (1-x)^2 (Beta(1,2)); v/(v+w) = 1 - r2 is uniform
    u = ba[0, :, 0].astype(np.float64)
    assert stats.kstest(u, lambda x: 1 - (1 - x) ** 2).pvalue > 1e-4
    vw = ba[0, :, 1] / (ba[0, :, 1] + ba[0, :, 2] + 1e-30)
    assert stats.kstest(vw[ba[0, :, 0] < 0.99], "uniform").pvalue > 1e-4
    # mean point tends to the area-weighted centroid of the surface
    cent = verts[0][faces].mean(axis=1)
    expect = (cent * A[:, None]).sum(0) / A.sum()
    assert np.all(np.abs(pts[0].mean(0) - expect) < 5e-3)


def test_points_lie_on_their_triangles():
    verts, faces = gen.trajectory(12, 3, 6)
    pts, fi, ba = oracle.sample_surface(verts, faces, 3000, seed=5)
    for t in range(3):
        P = verts[t][faces[fi[t]]].astype(np.float64)  # [N,3 corners,3]
        x = pts[t].astype(np.float64)
        e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
        nrm = np.cross(e1, e2)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        assert np.max(np.abs(((x - P[:, 0]) * nrm).sum(1))) < 1e-6
        # recover barycentrics by least squares in the triangle's plane
        M = np.stack([e1, e2], 2)
        sol = np.linalg.lstsq(M[0], (x - P[:, 0])[0], rcond=None)[0]
        lam = np.array([np.linalg.lstsq(M[k], (x - P[:, 0])[k], rcond=None)[0]
                        for k in range(0, 3000, 7)])
        assert sol.shape == (2,)
        assert lam.min() > -1e-5 and (lam.sum(1)).max() < 1 + 1e-5
        assert np.allclose(ba[t].sum(1), 1.0, atol=3e-7)


# ----------------------------------------------------------------- Chamfer
def test_chamfer_hand_example():
    g = GOLD["chamfer_two_to_one"]
    A = np.array(g["A"], np.float32)
    B = np.array(g["B"], np.float32)
    r1 = oracle.chamfer(A, B, 0)
    assert list(r1["idx_a"][0]) == g["idx_a"] and list(r1["idx_b"][0]) == g["idx_b"]
    assert r1["loss"][0] == g["eq1"]
    r2 = oracle.chamfer(A, B, 1)
    assert r2["loss"][0] == g["eq2"]
    gr = oracle.chamfer_grad(A, B, r1["idx_a"], r1["idx_b"], 0, want_b=True)
    assert np.array_equal(gr["ga"][0], np.array(g["grad_a_eq1"]))
    assert np.array_equal(gr["gb"][0], np.array(g["grad_b_eq1"]))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_nearest_matches_brute_force(seed):
    r = np.random.default_rng(seed)
    A = r.uniform(-0.5, 0.5, (11, 3)).astype(np.float32)
    B = r.uniform(-0.5, 0.5, (13, 3)).astype(np.float32)
    if seed % 2:
        B[7] = B[2]  # exact duplicate: ties go to the smaller index
        A[3] = B[5]
    idx, d32, d64 = oracle.nearest(A, B)
    bi, bd, bex = brute.nearest(A.tolist(), B.tolist())
    assert list(idx) == bi
    assert list(map(float, d32)) == bd
    for k in range(len(A)):
        assert abs(d64[k] - float(bex[k])) <= 4 * 2**-53 * float(bex[k])


def test_tie_break_smallest_index():
    B = np.array([[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0]], np.float32)
    A = np.zeros((1, 3), np.float32)
    idx, d32, _ = oracle.nearest(A, B)
    assert idx[0] == 0 and d32[0] == 1.0


def test_chamfer_invariants():
    r = np.random.default_rng(7)
    A = r.uniform(-0.5, 0.5, (300, 3)).astype(np.float32)
    B = r.uniform(-0.5, 0.5, (257, 3)).astype(np.float32)
    # zero for identical clouds, each point its own neighbour
    s = oracle.chamfer(A, A)
    assert s["loss"][0] == 0.0 and np.array_equal(s["idx_a"][0], np.arange(300))
    # Eq. 1 is symmetric, bit for bit
    ab = oracle.chamfer(A, B)["loss"][0]
    ba = oracle.chamfer(B, A)["loss"][0]
    assert ab == ba
    # scaling by 2 is exact: 4x loss, same neighbours
    s2 = oracle.chamfer(2 * A, 2 * B)
    s1 = oracle.chamfer(A, B)
    assert s2["loss"][0] == 4 * s1["loss"][0]
    assert np.array_equal(s2["idx_a"], s1["idx_a"]) and np.array_equal(s2["idx_b"], s1["idx_b"])
    # translation changes the loss only by rounding
    sh = np.array([0.125, -0.25, 0.0625], np.float32)
    st = oracle.chamfer(A + sh, B + sh)
    assert abs(st["loss"][0] - s1["loss"][0]) <= 1e-6 * s1["loss"][0]
    # permuting B permutes idx_a accordingly
    perm = r.permutation(257)
    sp = oracle.chamfer(A, B[perm])
    inv = np.argsort(perm)
    assert np.array_equal(perm[sp["idx_a"][0]], s1["idx_a"][0])
    assert np.array_equal(sp["idx_b"][0], s1["idx_b"][0][perm])
    assert inv.shape == perm.shape
    # Eq. 2 is the unnormalised sum of the first direction
    s_uni = oracle.chamfer(A, B, 1)
    assert abs(s_uni["loss"][0] - math.fsum(s1["d64a"][0])) <= 1e-12 * s_uni["loss"][0]


@pytest.mark.parametrize("reduction", [0, 1])
def test_chamfer_gradient_exact_differences(reduction):
    r = np.random.default_rng(11 + reduction)
    A = r.uniform(-0.5, 0.5, (6, 3)).astype(np.float32)
    B = r.uniform(-0.5, 0.5, (5, 3)).astype(np.float32)
    ch = oracle.chamfer(A, B, reduction)
    g = oracle.chamfer_grad(A, B, ch["idx_a"], ch["idx_b"], reduction)["ga"][0]
    ge = brute.grad_by_exact_differences(A.tolist(), B.tolist(), list(ch["idx_a"][0]),
                                         list(ch["idx_b"][0]), reduction)
    for i in range(6):
        for k in range(3):
            assert abs(g[i, k] - float(ge[i][k])) <= 1e-14 * (1 + abs(float(ge[i][k])))


def test_frame_weights_and_grad_scaling():
    r = np.random.default_rng(3)
    A = r.uniform(-0.5, 0.5, (3, 50, 3)).astype(np.float32)
    B = r.uniform(-0.5, 0.5, (3, 40, 3)).astype(np.float32)
    w = np.array([0.0, 1.0, 2.5], np.float32)
    base = oracle.chamfer(A, B, 0)
    wt = oracle.chamfer(A, B, 0, frame_w=w)
    assert np.allclose(wt["loss"], base["loss"] * w, rtol=1e-15, atol=0)
    g1 = oracle.chamfer_grad(A, B, base["idx_a"], base["idx_b"], 0)["ga"]
    gw = oracle.chamfer_grad(A, B, base["idx_a"], base["idx_b"], 0, frame_w=w,
                             grad_loss=np.array([3.0, 0.5, -2.0]))["ga"]
    for t, s in enumerate([0.0, 0.5, -5.0]):
        assert np.allclose(gw[t], g1[t] * s, rtol=1e-14, atol=0)


def test_vertex_gradient_matches_central_differences():
    verts, faces = gen.trajectory(6, 2, 3)
    obs = gen.observed_cloud(6, 2, 90, 3)
    pts, fi, ba = oracle.sample_surface(verts, faces, 80, seed=9)
    gv, gva, _ = oracle.full_gradient(verts, faces, obs, fi, ba, pts)
    coords = [(t, v, k) for t in range(2) for v in (0, 7, 20, 35) for k in range(3)]
    fd, fdz, moved = oracle.fd_gradient(verts, faces, obs, fi, ba, coords, h=1e-4)
    an = np.array([gv[t, v, k] for t, v, k in coords])
    # with neighbours frozen the loss is a quadratic in the vertices: central differences are
    # exact up to rounding.  The analytic gradient uses float points, the differences double
    # points, so allow the float rounding of the points.
    scale = np.array([gva[t, v, k] for t, v, k in coords]) + 1e-12
    assert np.all(np.abs(an - fdz) <= 1e-5 * scale + 1e-9)
    ok = ~moved
    assert np.all(np.abs(an[ok] - fd[ok]) <= 1e-5 * scale[ok] + 1e-9)


# ----------------------------------------------------------------- rigid bodies (Sec. III-C)
def test_rigid_rotation_matches_library_and_textbook():
    """[r] is Rz(psi) Ry(theta) Rx(phi): the images of the unit vectors are the columns of
    scipy's intrinsic 'ZYX' rotation, and quarter turns map axes as the textbook says."""
    from scipy.spatial.transform import Rotation
    p0 = np.eye(3, dtype=np.float32)
    starts = np.array([0, 3], np.int32)
    r = np.random.default_rng(5)
    for _ in range(20):
        phi, theta, psi = r.uniform(-np.pi, np.pi, 3)
        q = np.array([[[0, 0, 0, phi, theta, psi]]])
        cols = oracle.rigid_pose(q, p0, starts)[0]          # row j = R e_j
        R = Rotation.from_euler("ZYX", [psi, theta, phi]).as_matrix()
        assert np.allclose(cols.T, R, atol=1e-14)
    h = np.pi / 2
    ex, ey, ez = np.eye(3)
    img = lambda ang, v: oracle.rigid_pose(np.array([[[0, 0, 0, *ang]]]),
                                           v[None].astype(np.float32), np.array([0, 1], np.int32))[0, 0]
    assert np.allclose(img((h, 0, 0), ey), ez, atol=1e-15)   # roll about x
    assert np.allclose(img((0, h, 0), ez), ex, atol=1e-15)   # pitch about y
    assert np.allclose(img((0, 0, h), ex), ey, atol=1e-15)   # yaw about z
    # translation only
    t = oracle.rigid_pose(np.array([[[0.5, -1, 2, 0, 0, 0]]]), p0, starts)[0]
    assert np.array_equal(t, np.eye(3) + [0.5, -1, 2])


def test_rigid_pose_gradient_central_differences():
    """dL/dq for L(q) = sum_v g_v . p_v(q) against double central differences, two frames and
    three bodies covering part of the vertex range."""
    r = np.random.default_rng(8)
    V = 40
    p0 = r.normal(size=(V, 3)).astype(np.float32)
    starts = np.array([2, 15, 15, 33], np.int32)   # bodies of 13, 0 and 18 vertices
    q = r.uniform(-1, 1, (2, 3, 6))
    g = r.normal(size=(2, V, 3)).astype(np.float32)
    gq, ga = oracle.rigid_pose_grad(q, p0, starts, g)
    h = 1e-6
    for t in range(2):
        for b in range(3):
            for k in range(6):
                qp, qm = q.copy(), q.copy()
                qp[t, b, k] += h
                qm[t, b, k] -= h
                Lp = (oracle.rigid_pose(qp, p0, starts, V)[t] * g[t]).sum()
                Lm = (oracle.rigid_pose(qm, p0, starts, V)[t] * g[t]).sum()
                fd = (Lp - Lm) / (2 * h)
                assert abs(fd - gq[t, b, k]) <= 1e-7 * max(1.0, ga[t, b, k])
    assert np.all(gq[:, 1] == 0)                   # the empty body


def test_rigid_pose_gradient_special_cases():
    """A uniform gradient c on a body centred at its origin gives n c for the translation and
    zero for the angles; bad body ranges are rejected."""
    r = np.random.default_rng(9)
    half = r.normal(size=(15, 3)).astype(np.float32)
    p0 = np.concatenate([half, -half])            # points in +- pairs: an exact zero sum
    starts = np.array([0, 30], np.int32)
    c = np.array([0.25, -0.5, 2.0], np.float32)
    g = np.broadcast_to(c, (1, 30, 3)).copy()
    gq, ga = oracle.rigid_pose_grad(r.uniform(-1, 1, (1, 1, 6)), p0, starts, g)
    assert np.allclose(gq[0, 0, :3], 30 * c, rtol=1e-12)
    assert np.all(np.abs(gq[0, 0, 3:]) <= 1e-12 * ga[0, 0, 3:].max())
    with pytest.raises(oracle.OracleError):
        oracle.rigid_pose_grad(np.zeros((1, 1, 6)), p0, np.array([5, 3], np.int32), g)
