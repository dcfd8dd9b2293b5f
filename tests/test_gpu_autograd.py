"""The torch.autograd.Function over the C ABI: gradients against central finite differences of the
double-precision oracle loss, and against the oracle's analytic gradient (Sec. III-B Eq. 4 chained
with Eq. 1/2)."""
import numpy as np
import pytest

import oracle
from workloads import gen

from gpu_helpers import assert_grad, dev, gpu, host, say, torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_autograd_matches_finite_differences(precision):
    """4 frames of a 25x25 cloth, 2048 sampled vs 2048 observed points, loss summed over frames;
    d loss / d verts at 64 random vertices (all three axes, frame chosen per vertex) against
    (L(V+h e) - L(V-h e)) / 2h, h = 1e-4, in double with the face choice and weights fixed."""
    p = gpu()
    say(f"[autograd] FD precision={precision}")
    w = gen.workload(3)
    verts = dev(w["verts"]).requires_grad_(True)
    faces, obs = dev(w["faces"]), dev(w["observed"])
    loss = p.diffcloud_loss(verts, faces, obs, w["Na"], seed=w["seed"], precision=precision)
    loss.backward()
    g = host(verts.grad).astype(np.float64)
    # oracle: the same sampling (same counter-based words), double FD on the loss
    pts, fi, ba = oracle.sample_surface(w["verts"], faces=w["faces"], N=w["Na"], seed=w["seed"])
    och = oracle.chamfer(pts, w["observed"])
    assert abs(loss.item() - och["loss"].sum()) <= 1e-5 * och["loss"].sum()
    r = np.random.default_rng(3)
    verts_pick = gen.fd_vertices(w["V"], 64, 3)
    coords = [(int(r.integers(w["T"])), int(v), k) for v in verts_pick for k in range(3)]
    fd, fdz, moved = oracle.fd_gradient(w["verts"], w["faces"], w["observed"], fi, ba, coords,
                                        h=1e-4)
    ref = np.where(moved, fdz, fd)  # a neighbour change inside +-h: difference with frozen indices
    got = np.array([g[t, v, k] for t, v, k in coords])
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"[autograd] FD relative error {rel:.3e}, {int(moved.sum())} of {len(coords)} "
        "coordinates re-run with frozen neighbours")
    assert rel <= 1e-3
    # and the analytic double-precision gradient of the oracle, component by component
    ogv, ogva, _ = oracle.full_gradient(w["verts"], w["faces"], w["observed"], fi, ba, pts)
    assert_grad(g, ogv, ogva, what="autograd vs oracle")


def test_autograd_observed_gradient_and_weights():
    p = gpu()
    w = gen.workload(1)
    verts = dev(w["verts"]).requires_grad_(True)
    obs = dev(w["observed"]).requires_grad_(True)
    faces = dev(w["faces"])
    fw = dev(np.array([0.75], np.float32))
    out = p.DiffCloudChamfer.apply(verts, faces, obs, w["Na"], w["seed"], 0, 1, fw, None)
    (3.0 * out.sum()).backward()
    pts, fi, ba = oracle.sample_surface(w["verts"], w["faces"], w["Na"], seed=w["seed"])
    och = oracle.chamfer(pts, w["observed"], 1, np.array([0.75], np.float32))
    og = oracle.chamfer_grad(pts, w["observed"], och["idx_a"], och["idx_b"], 1,
                             np.array([0.75], np.float32), np.array([3.0]), want_b=True)
    assert_grad(host(obs.grad), og["gb"], og["gb_abs"], what="grad observed")
    ogv, ogva = oracle.sample_grad(og["ga"], w["faces"], fi, ba, w["V"], og["ga_abs"])
    assert_grad(host(verts.grad), ogv, ogva, what="grad verts")


def test_autograd_saves_indices_and_skips_recompute():
    """The backward uses the saved neighbours: running it twice gives bitwise the same gradient,
    and it launches no nearest-neighbour search (the all-pairs kernel count stays unchanged)."""
    p = gpu()
    w = gen.workload(3)
    ctx = p.default_context(0)
    verts = dev(w["verts"]).requires_grad_(True)
    faces, obs = dev(w["faces"]), dev(w["observed"])
    loss = p.diffcloud_loss(verts, faces, obs, w["Na"], seed=1)
    ctx.sync()
    ctx.kernel_times(reset=True)
    ctx.profile(True)
    g1 = torch.autograd.grad(loss, verts, retain_graph=True)[0].clone()
    g2 = torch.autograd.grad(loss, verts)[0]
    ctx.profile(False)
    kt = ctx.kernel_times(reset=True)
    assert kt["all_pairs"][1] == 0 and kt["backward"][1] == 4
    assert torch.equal(g1, g2)


@pytest.mark.parametrize("precision", [0, 1])
def test_autograd_unidirectional_loss(precision):
    """Eq. 2 (the loss the paper optimises) through the Function: only a -> b is searched, and the
    vertex gradient matches the oracle's analytic gradient of the summed Eq. 2 loss."""
    p = gpu()
    w = gen.workload(3)
    verts = dev(w["verts"]).requires_grad_(True)
    faces, obs = dev(w["faces"]), dev(w["observed"])
    loss = p.diffcloud_loss(verts, faces, obs, w["Na"], seed=w["seed"], precision=precision,
                            reduction=1)
    loss.backward()
    pts, fi, ba = oracle.sample_surface(w["verts"], faces=w["faces"], N=w["Na"], seed=w["seed"])
    ogv, ogva, och = oracle.full_gradient(w["verts"], w["faces"], w["observed"], fi, ba, pts,
                                          reduction=1)
    assert abs(loss.item() - och["loss"].sum()) <= 1e-5 * och["loss"].sum()
    assert_grad(host(verts.grad), ogv, ogva, what="Eq. 2 autograd vs oracle")


def test_autograd_masked_sampling():
    """Subset sampling through the Function: only faces of the mask receive points, so vertices
    touching no sampled face get exactly zero gradient; the gradient matches the oracle's."""
    p = gpu()
    w = gen.workload(3)
    faces_np = w["faces"]
    mask = (w["verts"][0][faces_np][:, :, 1].mean(axis=1) > 0).astype(np.uint8)
    verts = dev(w["verts"]).requires_grad_(True)
    faces, obs = dev(faces_np), dev(w["observed"])
    loss = p.diffcloud_loss(verts, faces, obs, w["Na"], seed=w["seed"], precision=1,
                            face_mask=torch.from_numpy(mask).to("cuda"))
    loss.backward()
    pts, fi, ba = oracle.sample_surface(w["verts"], faces=faces_np, N=w["Na"], seed=w["seed"],
                                        face_mask=mask)
    ogv, ogva, och = oracle.full_gradient(w["verts"], faces_np, w["observed"], fi, ba, pts)
    assert abs(loss.item() - och["loss"].sum()) <= 1e-5 * och["loss"].sum()
    g = host(verts.grad)
    assert_grad(g, ogv, ogva, what="masked autograd vs oracle")
    touched = np.zeros(w["V"], bool)
    touched[faces_np[mask == 1].ravel()] = True
    assert np.all(g[:, ~touched] == 0)
