"""The allocation-free sampling entry point (dc_sample_surface_noalloc, scratch in a static
device array) against dc_sample_surface: faces, points and barycentric weights bit for bit, on
two calls in a row (the second smaller, so that it starts from the first call's scratch
contents), without the context holding any scratch; too large a scratch is refused."""
import numpy as np
import pytest

from workloads import gen

from gpu_helpers import dev, gpu, host, say, torch

pytestmark = pytest.mark.gpu


def _outs(T, N):
    return (torch.empty((T, N, 3), dtype=torch.float32, device="cuda"),
            torch.empty((T, N), dtype=torch.int32, device="cuda"),
            torch.empty((T, N, 3), dtype=torch.float32, device="cuda"))


def test_sample_surface_noalloc_matches_sample_surface():
    p = gpu()
    ctx = p.Context(0)           # the allocation-free calls run on this one
    ref_ctx = p.Context(0)       # the existing entry point on its own context
    held0 = ctx.memory_held()[0]
    w4 = gen.workload(4)         # 100 frames of 19,602 faces: 15.7 MB of the 16 MiB scratch
    w2 = gen.workload(2, T=3)    # then a smaller call: 3 frames of 4,802 faces
    cases = [(w4, 4096, dict(seed=w4["seed"])),
             (w2, w2["Na"], dict(uniforms=dev(w2["words"].view(np.int32))))]
    for w, N, kw in cases:
        say(f"[no-alloc] {w['T']} frames, {w['F']} faces, {N} points, {sorted(kw)}")
        verts, faces = dev(w["verts"]), dev(w["faces"])
        out = _outs(w["T"], N)
        torch.cuda.synchronize()
        p.sample_surface_noalloc(verts, faces, N, out, ctx=ctx, **kw)
        ref = p.sample_surface(verts, faces, N, ctx=ref_ctx, **kw)
        torch.cuda.synchronize()
        ctx.sync()
        got = [host(x) for x in out]
        exp = [host(x) for x in ref]
        assert np.array_equal(got[1], exp[1])
        assert np.array_equal(got[0].view(np.uint32), exp[0].view(np.uint32))
        assert np.array_equal(got[2].view(np.uint32), exp[2].view(np.uint32))
        assert ctx.memory_held()[0] == held0  # the context took no scratch
    # a scratch beyond the static array is refused before any launch
    verts, faces = gen.trajectory(100, 110, 4)  # 110 frames of 19,602 faces: 17.2 MB
    out = _outs(110, 8)
    with pytest.raises(p.DCError) as e:
        p.sample_surface_noalloc(dev(verts), dev(faces), 8, out, seed=1, ctx=ctx)
    assert e.value.code == -6
    ctx.close()
    ref_ctx.close()
