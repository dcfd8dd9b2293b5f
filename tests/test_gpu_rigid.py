"""Rigid bodies (Sec. III-C): vertices from 6-DoF poses and the chain rule to the poses, against
the double-precision oracle, and the whole path pose -> vertices -> sampling -> Chamfer -> pose
gradient against central differences."""
import numpy as np
import pytest

import oracle
from workloads import gen

from gpu_helpers import dev, gpu, host, say, torch

pytestmark = pytest.mark.gpu


def _scene(seed=8, T=3, V=40):
    r = np.random.default_rng(seed)
    p0 = r.normal(size=(V, 3)).astype(np.float32)
    starts = np.array([2, 15, 15, 33], np.int32)   # bodies of 13, 0 and 18 vertices
    q = r.uniform(-1, 1, (T, 3, 6))
    return p0, starts, q


def test_rigid_pose_parity():
    """Each body vertex is the double-precision pose rounded once to float (within one ulp: the
    device's double sine and cosine may differ from the host's in the last bit); vertices owned
    by no body keep their values."""
    p = gpu()
    say("[rigid] pose parity")
    p0, starts, q = _scene()
    T, V = q.shape[0], p0.shape[0]
    base = torch.full((T, V, 3), 7.0, dtype=torch.float32, device="cuda")
    got = host(p.rigid_pose(dev(q), dev(p0), dev(starts), out=base))
    ref = oracle.rigid_pose(q, p0, starts, V)
    owned = np.zeros(V, bool)
    owned[2:33] = True
    r32 = ref[:, owned].astype(np.float32)
    ulp = np.spacing(np.abs(r32))
    assert np.all(np.abs(got[:, owned] - r32) <= ulp)
    assert np.all(got[:, ~owned] == 7.0)


def test_rigid_pose_gradient_parity():
    p = gpu()
    say("[rigid] pose gradient parity")
    p0, starts, q = _scene(9)
    g = np.random.default_rng(10).normal(size=(q.shape[0], p0.shape[0], 3)).astype(np.float32)
    got = host(p.rigid_pose_bwd(dev(q), dev(p0), dev(starts), dev(g)))
    ref, ref_abs = oracle.rigid_pose_grad(q, p0, starts, g)
    assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(ref_abs, 1e-300))
    assert np.all(got[:, 1] == 0)  # the empty body
    again = host(p.rigid_pose_bwd(dev(q), dev(p0), dev(starts), dev(g)))
    assert np.array_equal(got.view(np.uint64), again.view(np.uint64))


def test_rigid_bad_ranges():
    p = gpu()
    ctx = p.Context(0)
    p0, _, q = _scene()
    bad = dev(np.array([0, 20, 10, 40], np.int32))  # decreasing
    p.rigid_pose(dev(q), dev(p0), bad, ctx=ctx)
    with pytest.raises(p.DCError) as e:
        ctx.sync()
    assert e.value.code == -1
    over = dev(np.array([0, 20, 30, 41], np.int32))  # past V
    p.rigid_pose_bwd(dev(q), dev(p0), over, dev(np.zeros((3, 40, 3), np.float32)), ctx=ctx)
    with pytest.raises(p.DCError):
        ctx.sync()
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_rigid_chain_through_chamfer(precision):
    """A rigid 20x20 plate posed by q over two frames, sampled, compared with an observed cloud by
    Eq. 2: q.grad from autograd equals the oracle's chain (vertex gradient in double, then J^T)
    and the double central differences of the loss with face choice, weights and neighbours held
    fixed."""
    p = gpu()
    say(f"[rigid] chain through Chamfer precision={precision}")
    verts0, faces = gen.trajectory(20, 1, 6, sag=0.0)
    p0 = (verts0[0] - verts0[0].mean(0)).astype(np.float32)
    starts = np.array([0, p0.shape[0]], np.int32)
    T, N = 2, 1500
    q_np = np.array([[[0.02, -0.01, 0.03, 0.1, -0.05, 0.2]],
                     [[-0.03, 0.02, 0.0, -0.1, 0.08, -0.15]]])
    obs = gen.observed_cloud(20, T, N, 6, sag=0.0).astype(np.float32)  # stand-in observations
    q = dev(q_np).requires_grad_(True)
    verts = p.RigidPose.apply(q, dev(p0), dev(starts), None)
    loss = p.diffcloud_loss(verts, dev(faces), dev(obs), N, seed=77, precision=precision,
                            reduction=1)
    loss.backward()
    gq = host(q.grad)
    # the oracle's chain on the same float vertices: Eq. 4 + Chamfer gradient, then J^T
    v32 = host(verts.detach())
    pts, fi, ba = oracle.sample_surface(v32, faces, N, seed=77)
    gv, _, ch = oracle.full_gradient(v32, faces, obs, fi, ba, pts, reduction=1)
    ref, ref_abs = oracle.rigid_pose_grad(q_np, p0, starts, gv.astype(np.float32))
    assert np.all(np.abs(gq - ref) <= 1e-5 * np.maximum(ref_abs, 1e-12))
    # central differences in double, everything but the pose frozen
    ia = ch["idx_a"]
    h = 1e-6
    for t in range(T):
        for k in range(6):
            L = []
            for sgn in (1, -1):
                qq = q_np.copy()
                qq[t, 0, k] += sgn * h
                v64 = oracle.rigid_pose(qq, p0, starts)
                x64 = oracle.points_f64(v64[t:t + 1], faces, fi[t:t + 1], ba[t:t + 1])
                L.append(oracle.loss_f64(x64, obs[t:t + 1], 1, idx_a=ia[t:t + 1],
                                         idx_b=ch["idx_b"][t:t + 1]))
            fd = (L[0] - L[1]) / (2 * h)
            assert abs(fd - gq[t, 0, k]) <= 1e-4 * max(abs(fd), 1e-3 * np.abs(gq).max())
