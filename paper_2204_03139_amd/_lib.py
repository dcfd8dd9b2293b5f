"""ctypes binding of libdiffcloud.so: argument marshalling only.

Every function takes torch tensors that already live on the context's GPU, checks dtype, shape and
contiguity, and passes raw device pointers and the current HIP stream to the C ABI.  No
computation happens here.  If the library has not been built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdiffcloud.so")

DC_OK = 0
DC_PENDING = 1
DC_ERR_INVALID = -1
DC_ERR_NOMEM = -2
DC_ERR_BUDGET = -3
DC_ERR_HIP = -4
DC_ERR_DEGENERATE = -5
DC_ERR_UNSUPPORTED = -6

DC_PREC_FP32 = 0
DC_PREC_BF16_REFINE = 1
DC_RED_BIDIR_MEAN = 0
DC_RED_SIM2REAL_SUM = 1

STATUS_NAMES = {0: "DC_OK", 1: "DC_PENDING", -1: "DC_ERR_INVALID", -2: "DC_ERR_NOMEM",
                -3: "DC_ERR_BUDGET", -4: "DC_ERR_HIP", -5: "DC_ERR_DEGENERATE",
                -6: "DC_ERR_UNSUPPORTED"}

# every symbol the public header declares
EXPORTS = ["dc_create", "dc_destroy", "dc_last_error", "dc_sync", "dc_sample_surface",
           "dc_sample_surface_masked", "dc_area_cdf", "dc_rigid_pose", "dc_rigid_pose_bwd",
           "dc_sample_surface_bwd", "dc_chamfer_fwd", "dc_chamfer_bwd", "dc_get_stats",
           "dc_submit", "dc_poll", "dc_wait", "dc_version", "dc_debug_fail_allocs", "dc_profile",
           "dc_get_kernel_times", "dc_request_bytes", "dc_memory_held",
           "dc_sample_surface_noalloc"]


class DCError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("fallbacks", ctypes.c_uint64)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 4), ("launches", ctypes.c_uint64 * 4)]


KERNEL_CATEGORIES = ("all_pairs", "refine", "sampling", "backward")


class Request(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("faces", ctypes.c_void_p), ("T", ctypes.c_int),
                ("V", ctypes.c_int), ("F", ctypes.c_int), ("n_sim", ctypes.c_int),
                ("observed", ctypes.c_void_p), ("n_obs", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("precision", ctypes.c_int),
                ("reduction", ctypes.c_int), ("frame_w", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_void_p), ("grad_verts", ctypes.c_void_p),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("status", ctypes.c_int)]


_lib = None


def load():
    """Load the built library (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2204_03139_amd.build` "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
    L.dc_create.argtypes = [ctypes.POINTER(vp), i, ctypes.c_size_t, i]
    L.dc_destroy.argtypes = [vp]
    L.dc_last_error.argtypes = [vp]
    L.dc_last_error.restype = ctypes.c_char_p
    L.dc_sync.argtypes = [vp, vp]
    L.dc_sample_surface.argtypes = [vp, vp, vp, i, i, i, i, u64, vp, vp, vp, vp, vp]
    L.dc_sample_surface_masked.argtypes = [vp, vp, vp, i, i, i, i, u64, vp, vp, i, vp, vp, vp, vp]
    L.dc_sample_surface_noalloc.argtypes = [vp, vp, vp, i, i, i, i, u64, vp, vp, vp, vp, vp]
    L.dc_area_cdf.argtypes = [vp, vp, vp, i, i, i, vp, i, vp, vp, vp]
    L.dc_rigid_pose.argtypes = [vp, vp, vp, vp, i, i, i, vp, vp]
    L.dc_rigid_pose_bwd.argtypes = [vp, vp, vp, vp, vp, i, i, i, vp, vp]
    L.dc_sample_surface_bwd.argtypes = [vp, vp, vp, vp, vp, i, i, i, i, vp, vp]
    L.dc_chamfer_fwd.argtypes = [vp, vp, vp, i, i, i, i, i, vp, vp, vp, vp, vp, vp, vp]
    L.dc_chamfer_bwd.argtypes = [vp, vp, vp, vp, vp, vp, i, i, i, i, vp, vp, vp, vp]
    L.dc_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.dc_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(Result),
                            ctypes.POINTER(u64)]
    L.dc_poll.argtypes = [vp, u64]
    L.dc_wait.argtypes = [vp, u64, ctypes.c_int64]
    L.dc_request_bytes.argtypes = [ctypes.POINTER(Request), i, ctypes.POINTER(ctypes.c_size_t)]
    L.dc_debug_fail_allocs.argtypes = [vp, i]
    L.dc_memory_held.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_size_t)]
    L.dc_profile.argtypes = [vp, i]
    L.dc_get_kernel_times.argtypes = [vp, ctypes.POINTER(KernelTimes), i]
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc < 0:
        raise DCError(rc, where, load().dc_last_error(None).decode())
    return rc


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _words_ptr(u, shape):
    if u is None:
        return None
    return _ptr(u, u.dtype if u.dtype in (torch.int32, torch.uint32) else torch.int32, shape,
                "uniforms")


class Context:
    """A library context on one GPU (scratch memory, budget, serving loop)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, max_slots: int = 0):
        L = load()
        h = ctypes.c_void_p()
        _check(L.dc_create(ctypes.byref(h), device, hbm_budget_bytes, max_slots), "dc_create")
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load().dc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self, stream=None) -> int:
        return _check(load().dc_sync(self._h, _stream(stream)), "dc_sync")

    def stats(self) -> dict:
        st = Stats()
        _check(load().dc_get_stats(self._h, ctypes.byref(st)), "dc_get_stats")
        return dict(queries=st.queries, candidates=st.candidates, fallbacks=st.fallbacks)

    def profile(self, enable: bool = True):
        _check(load().dc_profile(self._h, int(enable)), "dc_profile")

    def kernel_times(self, reset: bool = True) -> dict:
        kt = KernelTimes()
        _check(load().dc_get_kernel_times(self._h, ctypes.byref(kt), int(reset)),
               "dc_get_kernel_times")
        return {name: (kt.ms[k], kt.launches[k]) for k, name in enumerate(KERNEL_CATEGORIES)}

    def memory_held(self) -> tuple[int, int]:
        """(device bytes held against the budget, the budget)."""
        held, budget = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().dc_memory_held(self._h, ctypes.byref(held), ctypes.byref(budget)),
               "dc_memory_held")
        return held.value, budget.value

    def debug_fail_allocs(self, n: int):
        _check(load().dc_debug_fail_allocs(self._h, n), "dc_debug_fail_allocs")


_default = {}


def default_context(device: int | None = None) -> Context:
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _default:
        _default[dev] = Context(dev)
    return _default[dev]


def sample_surface(verts, faces, N: int, seed: int = 0, uniforms=None, out=None, ctx=None,
                   stream=None, face_mask=None):
    """dc_sample_surface: returns (points [T,N,3], face_idx [T,N], bary [T,N,3]).  face_mask
    (uint8 [F] or [T,F], nonzero = may be drawn) selects dc_sample_surface_masked."""
    ctx = ctx or default_context(verts.device.index)
    T, V, _ = verts.shape
    F = faces.shape[0]
    if out is None:
        points = torch.empty((T, N, 3), dtype=torch.float32, device=verts.device)
        face_idx = torch.empty((T, N), dtype=torch.int32, device=verts.device)
        bary = torch.empty((T, N, 3), dtype=torch.float32, device=verts.device)
    else:
        points, face_idx, bary = out
    outs = (_ptr(points, torch.float32, (T, N, 3), "points"),
            _ptr(face_idx, torch.int32, (T, N), "face_idx"),
            _ptr(bary, torch.float32, (T, N, 3), "bary"), _stream(stream))
    ins = (ctx.handle, _ptr(verts, torch.float32, (T, V, 3), "verts"),
           _ptr(faces, torch.int32, (F, 3), "faces"), T, V, F, N, seed & (2**64 - 1),
           _words_ptr(uniforms, (T, N, 4)))
    if face_mask is None:
        rc = load().dc_sample_surface(*ins, *outs)
        _check(rc, "dc_sample_surface")
    else:
        per_frame = face_mask.dim() == 2
        m = _ptr(face_mask, torch.uint8, (T, F) if per_frame else (F,), "face_mask")
        rc = load().dc_sample_surface_masked(*ins, m, int(per_frame), *outs)
        _check(rc, "dc_sample_surface_masked")
    return points, face_idx, bary


def area_cdf(verts, faces, face_mask=None, out=None, ctx=None, stream=None):
    """dc_area_cdf: returns (cdf [T,F] float64, last_face [T] int32) of the mesh (verts [T,V,3],
    faces [F,3]); face_mask (uint8 [F] or [T,F]) restricts the faces as in sample_surface."""
    ctx = ctx or default_context(verts.device.index)
    T, V, _ = verts.shape
    F = faces.shape[0]
    if out is None:
        cdf = torch.empty((T, F), dtype=torch.float64, device=verts.device)
        last = torch.empty((T,), dtype=torch.int32, device=verts.device)
    else:
        cdf, last = out
    per_frame = face_mask is not None and face_mask.dim() == 2
    m = None if face_mask is None else _ptr(face_mask, torch.uint8, (T, F) if per_frame else (F,),
                                            "face_mask")
    rc = load().dc_area_cdf(ctx.handle, _ptr(verts, torch.float32, (T, V, 3), "verts"),
                            _ptr(faces, torch.int32, (F, 3), "faces"), T, V, F, m, int(per_frame),
                            _ptr(cdf, torch.float64, (T, F), "cdf"),
                            _ptr(last, torch.int32, (T,), "last_face"), _stream(stream))
    _check(rc, "dc_area_cdf")
    return cdf, last


def sample_surface_noalloc(verts, faces, N: int, out, seed: int = 0, uniforms=None, ctx=None,
                           stream=None):
    """dc_sample_surface_noalloc: sampling into the caller's `out` = (points [T,N,3],
    face_idx [T,N], bary [T,N,3]) with the library allocating nothing (its scratch is a static
    device array); returns `out`."""
    ctx = ctx or default_context(verts.device.index)
    T, V, _ = verts.shape
    F = faces.shape[0]
    points, face_idx, bary = out
    rc = load().dc_sample_surface_noalloc(
        ctx.handle, _ptr(verts, torch.float32, (T, V, 3), "verts"),
        _ptr(faces, torch.int32, (F, 3), "faces"), T, V, F, N, seed & (2**64 - 1),
        _words_ptr(uniforms, (T, N, 4)), _ptr(points, torch.float32, (T, N, 3), "points"),
        _ptr(face_idx, torch.int32, (T, N), "face_idx"),
        _ptr(bary, torch.float32, (T, N, 3), "bary"), _stream(stream))
    _check(rc, "dc_sample_surface_noalloc")
    return out


def sample_surface_bwd(grad_points, faces, face_idx, bary, V: int, out=None, ctx=None,
                       stream=None):
    ctx = ctx or default_context(grad_points.device.index)
    T, N, _ = grad_points.shape
    F = faces.shape[0]
    gv = out if out is not None else torch.empty((T, V, 3), dtype=torch.float32,
                                                 device=grad_points.device)
    rc = load().dc_sample_surface_bwd(
        ctx.handle, _ptr(grad_points, torch.float32, (T, N, 3), "grad_points"),
        _ptr(faces, torch.int32, (F, 3), "faces"), _ptr(face_idx, torch.int32, (T, N), "face_idx"),
        _ptr(bary, torch.float32, (T, N, 3), "bary"), T, V, F, N,
        _ptr(gv, torch.float32, (T, V, 3), "grad_verts"), _stream(stream))
    _check(rc, "dc_sample_surface_bwd")
    return gv


def chamfer_fwd(a, b, precision: int = DC_PREC_FP32, reduction: int = DC_RED_BIDIR_MEAN,
                frame_w=None, out=None, ctx=None, stream=None, b_side: bool = True):
    """dc_chamfer_fwd: returns dict(dist_a, idx_a, dist_b, idx_b, loss).  With the
    unidirectional reduction, b_side=False searches only a -> b (dist_b, idx_b are None)."""
    ctx = ctx or default_context(a.device.index)
    T, Na, _ = a.shape
    Nb = b.shape[1]
    dev = a.device
    if out is None:
        out = dict(dist_a=torch.empty((T, Na), dtype=torch.float32, device=dev),
                   idx_a=torch.empty((T, Na), dtype=torch.int32, device=dev),
                   dist_b=torch.empty((T, Nb), dtype=torch.float32, device=dev) if b_side else None,
                   idx_b=torch.empty((T, Nb), dtype=torch.int32, device=dev) if b_side else None,
                   loss=torch.empty((T,), dtype=torch.float64, device=dev))
    rc = load().dc_chamfer_fwd(
        ctx.handle, _ptr(a, torch.float32, (T, Na, 3), "a"), _ptr(b, torch.float32, (T, Nb, 3), "b"),
        T, Na, Nb, precision, reduction, _ptr(frame_w, torch.float32, (T,), "frame_w"),
        _ptr(out["dist_a"], torch.float32, (T, Na), "dist_a"),
        _ptr(out["idx_a"], torch.int32, (T, Na), "idx_a"),
        _ptr(out["dist_b"], torch.float32, (T, Nb), "dist_b"),
        _ptr(out["idx_b"], torch.int32, (T, Nb), "idx_b"),
        _ptr(out["loss"], torch.float64, (T,), "loss"), _stream(stream))
    _check(rc, "dc_chamfer_fwd")
    return out


def chamfer_bwd(grad_loss, a, b, idx_a, idx_b, reduction: int = DC_RED_BIDIR_MEAN, frame_w=None,
                want_b: bool = False, out=None, ctx=None, stream=None):
    """dc_chamfer_bwd: returns (grad_a [T,Na,3], grad_b [T,Nb,3] or None)."""
    ctx = ctx or default_context(a.device.index)
    T, Na, _ = a.shape
    Nb = b.shape[1]
    if out is None:
        ga = torch.empty((T, Na, 3), dtype=torch.float32, device=a.device)
        gb = torch.empty((T, Nb, 3), dtype=torch.float32, device=a.device) if want_b else None
    else:
        ga, gb = out
    rc = load().dc_chamfer_bwd(
        ctx.handle, _ptr(grad_loss, torch.float64, (T,), "grad_loss"),
        _ptr(a, torch.float32, (T, Na, 3), "a"), _ptr(b, torch.float32, (T, Nb, 3), "b"),
        _ptr(idx_a, torch.int32, (T, Na), "idx_a"), _ptr(idx_b, torch.int32, (T, Nb), "idx_b"),
        T, Na, Nb, reduction, _ptr(frame_w, torch.float32, (T,), "frame_w"),
        _ptr(ga, torch.float32, (T, Na, 3), "grad_a"),
        _ptr(gb, torch.float32, (T, Nb, 3), "grad_b"), _stream(stream))
    _check(rc, "dc_chamfer_bwd")
    return ga, gb


def rigid_pose(q, p0, body_start, out=None, ctx=None, stream=None):
    """dc_rigid_pose: vertices [T,V,3] of rigid bodies at poses q [T,B,6] (float64).  Vertices
    owned by no body keep the values of `out` (uninitialised when out is None)."""
    ctx = ctx or default_context(q.device.index)
    T, B, _ = q.shape
    V = p0.shape[0]
    verts = out if out is not None else torch.empty((T, V, 3), dtype=torch.float32, device=q.device)
    rc = load().dc_rigid_pose(
        ctx.handle, _ptr(q, torch.float64, (T, B, 6), "q"), _ptr(p0, torch.float32, (V, 3), "p0"),
        _ptr(body_start, torch.int32, (B + 1,), "body_start"), T, B, V,
        _ptr(verts, torch.float32, (T, V, 3), "verts"), _stream(stream))
    _check(rc, "dc_rigid_pose")
    return verts


def rigid_pose_bwd(q, p0, body_start, grad_verts, out=None, ctx=None, stream=None):
    """dc_rigid_pose_bwd: the pose gradient [T,B,6] (float64)."""
    ctx = ctx or default_context(q.device.index)
    T, B, _ = q.shape
    V = p0.shape[0]
    gq = out if out is not None else torch.empty((T, B, 6), dtype=torch.float64, device=q.device)
    rc = load().dc_rigid_pose_bwd(
        ctx.handle, _ptr(q, torch.float64, (T, B, 6), "q"), _ptr(p0, torch.float32, (V, 3), "p0"),
        _ptr(body_start, torch.int32, (B + 1,), "body_start"),
        _ptr(grad_verts, torch.float32, (T, V, 3), "grad_verts"), T, B, V,
        _ptr(gq, torch.float64, (T, B, 6), "grad_q"), _stream(stream))
    _check(rc, "dc_rigid_pose_bwd")
    return gq
