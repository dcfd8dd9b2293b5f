// Allocation-free sampling: dc_sample_surface with its scratch (the per-frame area CDF in double
// and the last drawable face of each frame, Sec. III-B) in a static device array, for callers
// that cannot allocate device memory.  The kernels are those of dc_sample_surface.
#include <mutex>

#include "batch.h"

namespace dc {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;

// The scratch of dc_sample_surface_noalloc: one copy per GPU, held until the process ends.  In
// host code this name is not a device address; each device's address comes from
// hipGetSymbolAddress in noalloc_init.
__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

char *scratch_ptr(int device) {
    std::lock_guard<std::mutex> g(g_mu);
    return (device >= 0 && device < MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace

// Once per device, with that device current: the device address of `scratch` on it.
int noalloc_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("device index beyond the allocation-free scratch table");
        return DC_ERR_INVALID;
    }
    std::lock_guard<std::mutex> g(g_mu);
    if (g_scratch_ptr[device]) return DC_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) {
        set_error("hipGetSymbolAddress(scratch) returned NULL");
        return DC_ERR_HIP;
    }
    g_scratch_ptr[device] = static_cast<char *>(p);
    return DC_OK;
}

}  // namespace dc

using namespace dc;

extern "C" int dc_sample_surface_noalloc(dc_ctx *ctx, const float *verts, const int32_t *faces,
                                         int T, int V, int F, int N, uint64_t seed,
                                         const uint32_t *uniforms, float *points,
                                         int32_t *face_idx, float *bary, void *stream) {
    clear_error();
    if (!ctx || !verts || !faces || !points || !face_idx || !bary) {
        set_error("dc_sample_surface_noalloc: NULL argument");
        return DC_ERR_INVALID;
    }
    if (T < 1 || T > 65535 || V < 1 || V > (1 << 24) || F < 1 || F > (1 << 24) || N < 1 ||
        N > (1 << 24)) {
        set_error("dc_sample_surface_noalloc: T must be in [1, 65535] and V, F, N in [1, 2^24]");
        return DC_ERR_INVALID;
    }
    const size_t cdf_bytes = Arena::need((size_t)T * F, sizeof(double));
    const size_t need = sample_scratch_bytes(T, F);
    if (need > NOALLOC_SCRATCH_BYTES) {
        set_error("dc_sample_surface_noalloc: " + std::to_string(T) + " frames of " +
                  std::to_string(F) + " faces need " + std::to_string(need) +
                  " bytes of scratch, more than its " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                  " bytes");
        return DC_ERR_UNSUPPORTED;
    }
    char *base = scratch_ptr(ctx->device);
    if (!base) {
        set_error("dc_sample_surface_noalloc: the scratch address of this device is unknown");
        return DC_ERR_HIP;
    }
    DC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->mu);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    launch_sample(verts, faces, T, V, F, N, seed, uniforms, nullptr, 0, points, face_idx, bary,
                  reinterpret_cast<double *>(base), reinterpret_cast<int32_t *>(base + cdf_bytes),
                  ctx->d_status, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "sample_surface_noalloc launch");
    return DC_OK;
}
