"""The synthetic input recipe (CPU): observed clouds are spread uniformly over the area of the
mesh surface, whatever its slopes."""
import numpy as np
from scipy import stats

from workloads import gen


def test_observed_points_are_area_uniform_on_the_surface():
    """Points of the rejection sampler (before noise) per grid triangle against the triangles'
    3-D areas: chi-square at 1e-3, on a steep surface where uniform (x, y) draws would be far off
    (they would follow the projected areas, all equal)."""
    n = 9
    xy, faces = gen.grid_mesh(n)
    z = 0.25 * np.sin(2 * np.pi * 1.5 * xy[:, 0]) * np.cos(2 * np.pi * xy[:, 1])
    zgrid = z.reshape(n, n)
    rng = np.random.default_rng(5)
    count = 200_000
    x, y, zz = gen._surface_uniform_xy(rng, zgrid, n, count)
    assert len(x) == count
    # which triangle each point is in (lower: s >= r), as in the grid's face order
    gx, gy = (x + 0.5) * (n - 1), (y + 0.5) * (n - 1)
    i = np.clip(np.floor(gx).astype(int), 0, n - 2)
    j = np.clip(np.floor(gy).astype(int), 0, n - 2)
    upper = (gx - i) < (gy - j)
    tri = 2 * (j * (n - 1) + i) + upper
    counts = np.bincount(tri, minlength=len(faces))
    P = np.c_[xy, z]
    e1 = P[faces[:, 1]] - P[faces[:, 0]]
    e2 = P[faces[:, 2]] - P[faces[:, 0]]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
    expected = count * area / area.sum()
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert stats.chi2.sf(chi2, len(faces) - 1) > 1e-3
    # and the points lie on the surface
    zs, _ = gen._grid_cell(zgrid, n, x, y)
    assert np.array_equal(zs, zz)
    # the surface is steep enough that projected-area (uniform x, y) draws would fail the test:
    # the same chi-square against equal expected counts rejects
    assert area.max() / area.min() > 1.5
    even = np.full(len(faces), count / len(faces))
    assert stats.chi2.sf(((counts - even) ** 2 / even).sum(), len(faces) - 1) < 1e-6
