"""GPU parity of the face areas and their running sum (Sec. III-B, Eq. 3: the table the
area-weighted face choice is drawn from) through dc_area_cdf: every C_k bit for bit equal to the
oracle's plain left-to-right double sum of the oracle's areas, and the last face of positive area.

The device adds the areas of a binade in parallel (rounding each area to the binade's grid) and
falls back to one ordinary addition at ties and binade changes; the inputs below are built so that
every one of those paths is taken: exact ties in both rounding directions, jumps over many
binades, leading and interleaved zero areas, non-finite areas, and sizes around the window
(960 areas) and chunk (4,000 areas) boundaries."""
import numpy as np
import pytest

import oracle
from workloads import gen

from gpu_helpers import dev, gpu, host, say, torch

pytestmark = pytest.mark.gpu


def _expected(verts, faces, mask=None):
    """Oracle CDF [T,F], last drawable face [T] (-1 for a degenerate frame), degenerate flags."""
    T, F = verts.shape[0], faces.shape[0]
    C = np.zeros((T, F))
    last = np.full(T, -1, np.int32)
    degenerate = []
    for t in range(T):
        A = oracle.face_areas(verts[t], faces)
        if mask is not None:
            A[(mask[t] if mask.ndim == 2 else mask) == 0] = 0.0
        C[t], rc = oracle.area_cdf(A)
        pos = np.nonzero(A > 0)[0]
        if rc == 0 and len(pos):
            last[t] = pos[-1]
        degenerate.append(rc != 0)
    return C, last, degenerate


def _check(p, verts, faces, mask=None, what=""):
    say(f"[area_cdf] {what} T={verts.shape[0]} F={faces.shape[0]}")
    ctx = p.Context(0)
    m = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask)).to("cuda")
    cdf, last = p.area_cdf(dev(verts), dev(faces), face_mask=m, ctx=ctx)
    C, L, degenerate = _expected(verts, faces, mask)
    if any(degenerate):
        with pytest.raises(p.DCError) as e:
            ctx.sync()
        assert e.value.code == -5
    else:
        ctx.sync()
    ctx.close()
    got = host(cdf)
    nan_g, nan_e = np.isnan(got), np.isnan(C)
    assert np.array_equal(nan_g, nan_e), f"{what}: NaN positions differ"
    bad = (got.view(np.uint64) != C.view(np.uint64)) & ~nan_e
    assert not bad.any(), f"{what}: {bad.sum()} sums differ, first at {np.argwhere(bad)[0]}"
    assert np.array_equal(host(last), L), f"{what}: last faces differ"
    return C


def _tie_count(A, C):
    """Additions of one run whose exact sum lies halfway between two doubles."""
    prev = np.concatenate([[0.0], C[:-1]])
    ok = (prev > 0) & np.isfinite(prev) & np.isfinite(A)
    u = np.spacing(prev[ok])
    frac = np.mod(A[ok] / u, 1.0)
    return int(np.sum(frac == 0.5))


def _tie_mesh(F, seed):
    """A big triangle of area 2^40, then right triangles of area k 2^-14 (k = 0..7) in random
    order: against the sum's spacing 2^-12 their areas are k/4 of a step, so k = 2 and 6 are ties
    whose direction depends on the running sum; later a second big triangle moves the sum up
    one binade, where k = 4 becomes the tie."""
    rng = np.random.default_rng(seed)
    v = [[0, 0, 0], [2.0 ** 20, 0, 0], [0, 2.0 ** 21, 0], [0, 0, 1], [2.0 ** -7, 0, 1]]
    v += [[0, k * 2.0 ** -6, 1] for k in range(1, 8)]
    ks = rng.integers(0, 8, F)
    faces = np.array([[3, 4, 4 + k] if k else [3, 4, 3] for k in ks], np.int32)
    faces[0] = [0, 1, 2]
    faces[F // 2] = [0, 1, 2]
    verts = np.array(v, np.float32)[None]
    return verts, faces


def test_grid_frames():
    """The 100x100 cloth of the headline workload (19,602 faces: five chunks) and a small one."""
    p = gpu()
    verts, faces = gen.trajectory(100, 2, 4)
    _check(p, verts, faces, what="grid 100")
    verts, faces = gen.trajectory(25, 3, 1)
    _check(p, verts, faces, what="grid 25")


@pytest.mark.parametrize("seed", [0, 1])
def test_ties_and_binade_changes(seed):
    p = gpu()
    verts, faces = _tie_mesh(9000, seed)
    C = _check(p, verts, faces, what=f"ties seed {seed}")
    ties = _tie_count(oracle.face_areas(verts[0], faces), C[0])
    assert ties > 1000, f"the mesh should produce many ties, got {ties}"


def test_wide_range_of_areas():
    """Areas from 1e-40 to 1e36 in random order: sums jump over many binades at once."""
    p = gpu()
    rng = np.random.default_rng(7)
    F = 6000
    scale = 10.0 ** rng.uniform(-20, 18, F)
    base = rng.uniform(-1, 1, (F, 3, 3)) * scale[:, None, None]
    verts = base.reshape(1, 3 * F, 3).astype(np.float32)
    faces = np.arange(3 * F, dtype=np.int32).reshape(F, 3)
    _check(p, verts, faces, what="wide range")


def test_masks_with_leading_and_interleaved_zeros():
    p = gpu()
    verts, faces = gen.trajectory(60, 3, 2)
    F = len(faces)
    mask = np.ones((3, F), np.uint8)
    mask[0, : int(0.7 * F)] = 0                      # a long run of zeros before the first area
    mask[1] = (np.arange(F) // 513) % 2              # runs of 513 zeros, across windows
    mask[2] = np.random.default_rng(3).random(F) < 0.05  # sparse areas between zeros
    _check(p, verts, faces, mask=mask, what="masks")
    _check(p, verts[:1], faces, mask=mask[0], what="shared mask")


def test_non_finite_and_zero_frames():
    """A NaN vertex makes the sums NaN from its first face on; an infinite coordinate gives
    infinite and NaN areas; a flat frame has zero sums.  All three frames are degenerate."""
    p = gpu()
    verts, faces = gen.trajectory(40, 4, 2)
    verts = verts.copy()
    verts[0, 500] = np.nan
    verts[1, 300] = [np.inf, 0.0, 0.0]  # infinite (and NaN) areas around one vertex
    verts[2] = 0.5                       # every face has zero area
    _check(p, verts, faces, what="non-finite")


@pytest.mark.parametrize("F", [1, 2, 959, 961, 1025, 3999, 4000, 4001, 8193])
def test_sizes_around_windows_and_chunks(F):
    p = gpu()
    rng = np.random.default_rng(F)
    verts = rng.uniform(-1, 1, (2, 3 * F, 3)).astype(np.float32)
    faces = rng.permutation(3 * F).astype(np.int32).reshape(F, 3)
    _check(p, verts, faces, what=f"F={F}")


def test_many_chunks():
    """A frame of 1,000,003 faces (250 chunks of 4,000, the last one ragged) with areas over six
    orders of magnitude, and a second frame with every tenth face masked."""
    p = gpu()
    rng = np.random.default_rng(11)
    F = 1_000_003
    scale = 10.0 ** rng.uniform(-3, 0, F)
    base = rng.uniform(-1, 1, (F, 3, 3)) * scale[:, None, None]
    verts = np.stack([base.reshape(3 * F, 3), base[::-1].reshape(3 * F, 3)]).astype(np.float32)
    faces = np.arange(3 * F, dtype=np.int32).reshape(F, 3)
    mask = np.ones((2, F), np.uint8)
    mask[1, ::10] = 0
    _check(p, verts, faces, mask=mask, what="many chunks")


def test_bad_face_and_arguments():
    p = gpu()
    ctx = p.Context(0)
    verts, faces = gen.trajectory(10, 1, 1)
    faces = faces.copy()
    faces[7, 1] = verts.shape[1]  # names a vertex that does not exist
    cdf, last = p.area_cdf(dev(verts), dev(faces), ctx=ctx)
    with pytest.raises(p.DCError) as e:
        ctx.sync()
    assert e.value.code == -1
    assert host(last)[0] == -1
    with pytest.raises(ValueError):  # wrong mask shape
        p.area_cdf(dev(verts), dev(faces), ctx=ctx,
                   face_mask=torch.ones(len(faces) + 1, dtype=torch.uint8, device="cuda"))
    ctx.close()
