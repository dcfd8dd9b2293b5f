"""The allocation-free sampling entry point under HIP graph capture (the callers it is for): a
captured call replayed several times, with eager work and synchronisation between the replays and
new vertex positions written into the captured input each time, equals an eager call of
dc_sample_surface on the same inputs, bit for bit, on every replay."""
import numpy as np
import pytest

from workloads import gen

from gpu_helpers import dev, gpu, host, say, torch

pytestmark = pytest.mark.gpu


def test_noalloc_sampling_replays_in_a_graph():
    p = gpu()
    say("[graph] capture and replay of dc_sample_surface_noalloc")
    ctx = p.Context(0)
    w = gen.workload(2, T=3)
    T, N = w["T"], w["Na"]
    verts = dev(w["verts"])
    faces = dev(w["faces"])
    out = (torch.empty((T, N, 3), dtype=torch.float32, device="cuda"),
           torch.empty((T, N), dtype=torch.int32, device="cuda"),
           torch.empty((T, N, 3), dtype=torch.float32, device="cuda"))
    # warm the entry point up once outside the capture
    p.sample_surface_noalloc(verts, faces, N, out, seed=w["seed"], ctx=ctx)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p.sample_surface_noalloc(verts, faces, N, out, seed=w["seed"], ctx=ctx)
    r = np.random.default_rng(3)
    for k in range(4):
        # new positions in the captured input buffer, some eager work between replays
        verts.copy_(dev(w["verts"] + r.normal(0, 0.01, w["verts"].shape).astype(np.float32)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = p.sample_surface(verts, faces, N, seed=w["seed"], ctx=ctx)
        torch.cuda.synchronize()
        ctx.sync()
        for a, b in zip(out, ref):
            assert np.array_equal(host(a).view(np.uint8), host(b).view(np.uint8)), k
    ctx.close()
