// C ABI entry points of libdiffcloud: argument validation, scratch management under the HBM
// budget, and the launch sequence of each call.  Every kernel runs on the caller's stream.
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "batch.h"
#include "scheduler.h"

namespace dc {

static thread_local std::string g_err;
thread_local Recording *g_record = nullptr;

void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

int hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return DC_ERR_HIP;
}

int budget_take(dc_ctx *ctx, size_t bytes) {
    std::lock_guard<std::mutex> g(ctx->budget_mu);
    if (ctx->held + bytes > ctx->budget) {
        set_error("HBM budget exceeded: need " + std::to_string(bytes) + " bytes, " +
                  std::to_string(ctx->budget - ctx->held) + " free");
        return DC_ERR_BUDGET;
    }
    ctx->held += bytes;
    return DC_OK;
}

void budget_give(dc_ctx *ctx, size_t bytes) {
    std::lock_guard<std::mutex> g(ctx->budget_mu);
    ctx->held -= bytes;
}

bool forced_alloc_failure(dc_ctx *ctx) {
    std::lock_guard<std::mutex> g(ctx->budget_mu);
    if (ctx->fail_next_alloc <= 0) return false;
    --ctx->fail_next_alloc;
    return true;
}

int dev_alloc_raw(dc_ctx *ctx, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return DC_OK;
    int rc = budget_take(ctx, bytes);
    if (rc != DC_OK) return rc;
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        budget_give(ctx, bytes);
        *p = nullptr;
        set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
        return DC_ERR_NOMEM;
    }
    return DC_OK;
}

int dev_alloc(dc_ctx *ctx, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return DC_OK;
    if (forced_alloc_failure(ctx)) {
        set_error("device allocation of " + std::to_string(bytes) + " bytes failed (forced)");
        return DC_ERR_NOMEM;
    }
    return dev_alloc_raw(ctx, p, bytes);
}

void dev_free(dc_ctx *ctx, void *p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    budget_give(ctx, bytes);
}

int arena_reserve(dc_ctx *ctx, size_t bytes, hipStream_t s) {
    if (ctx->arena_used && s != ctx->arena_stream)
        DC_HIP(hipStreamWaitEvent(s, ctx->arena_ev, 0));
    Arena &a = ctx->arena;
    a.reset();
    if (bytes <= a.cap) return DC_OK;
    // the old buffer may still be read by queued work: wait for the device before freeing it
    DC_HIP(hipDeviceSynchronize());
    dev_free(ctx, a.base, a.cap);
    a.base = nullptr;
    a.cap = 0;
    const size_t want = (bytes + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
    void *p = nullptr;
    int rc = dev_alloc(ctx, &p, want);
    if (rc != DC_OK) return rc;
    a.base = static_cast<char *>(p);
    a.cap = want;
    return DC_OK;
}

ArenaUse::~ArenaUse() {
    if (hipEventRecord(ctx->arena_ev, s) == hipSuccess) {
        ctx->arena_stream = s;
        ctx->arena_used = true;
    } else {
        // without a record the next call cannot order itself after this one: wait here instead
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        ctx->arena_used = false;
    }
}

static int check_dims(int T, std::initializer_list<long> sizes) {
    if (T < 1 || T > 65535) {
        set_error("T must be in [1, 65535]");
        return DC_ERR_INVALID;
    }
    for (long n : sizes)
        if (n < 1 || n > (1L << 24)) {
            set_error("sizes must be in [1, 2^24]");
            return DC_ERR_INVALID;
        }
    return DC_OK;
}

static int launched(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return DC_OK;
}

// Shared by the direct calls and the serving loop: sampling with its scratch carved from `ar`.
ProfScope::ProfScope(dc_ctx *c, int category, hipStream_t st) : ctx(c), cat(category), s(st) {
    if (!ctx || !ctx->prof || hipEventCreate(&a) != hipSuccess) {
        ctx = nullptr;
        return;
    }
    (void)hipEventRecord(a, s);
}

ProfScope::~ProfScope() {
    if (!ctx) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> g(ctx->prof_mu);
    ctx->prof_pending.push_back({cat, a, b});
}

int enqueue_sample(dc_ctx *prof, const float *verts, const int32_t *faces, int T, int V, int F,
                   int N, uint64_t seed, const uint32_t *uniforms, const uint8_t *mask,
                   int mask_per_frame, float *points, int32_t *face_idx, float *bary, Arena &ar,
                   unsigned *status, hipStream_t s) {
    double *cdf = ar.take<double>((size_t)T * F);
    int32_t *lastpos = ar.take<int32_t>((size_t)T);
    ProfScope ps(prof, 2, s);
    launch_sample(verts, faces, T, V, F, N, seed, uniforms, mask, mask_per_frame, points,
                  face_idx, bary, cdf, lastpos, status, s);
    return launched("sample_surface launch");
}

size_t chamfer_fwd_scratch_bytes(int T, int Na, int Nb, int precision) {
    if (precision == DC_PREC_BF16_REFINE) return screen_scratch_bytes(T, Na, Nb);
    return std::max({nn_exact_scratch_bytes(T, Na, Nb), nn_exact_scratch_bytes(T, Nb, Na),
                     nn_bidir_scratch_bytes(T, Na, Nb)});
}

int enqueue_chamfer_fwd(dc_ctx *prof, const float *a, const float *b, int T, int Na, int Nb,
                        int precision, int reduction, const float *frame_w, float *dist_a,
                        int32_t *idx_a, float *dist_b, int32_t *idx_b, double *loss,
                        char *scratch, unsigned long long *stats, hipStream_t s) {
    // idx_b == NULL: the unidirectional loss (Eq. 2) needs only the a -> b direction
    if (precision == DC_PREC_BF16_REFINE) {
        launch_chamfer_screened(a, Na, b, Nb, T, idx_a, dist_a, idx_b, dist_b, scratch, stats,
                                prof, s);
    } else {
        // both directions: one pass over the pairs when the frames are large enough
        bool done = false;
        if (idx_b) {
            ProfScope ps(prof, 0, s);
            done = launch_nn_bidir(a, Na, b, Nb, T, idx_a, dist_a, idx_b, dist_b, scratch, s);
        }
        if (!done) {
            {
                ProfScope ps(prof, 0, s);
                launch_nn_exact_ws(a, Na, b, Nb, T, idx_a, dist_a, scratch, s);
            }
            if (idx_b) {
                ProfScope ps(prof, 0, s);
                launch_nn_exact_ws(b, Nb, a, Na, T, idx_b, dist_b, scratch, s);
            }
        }
    }
    launch_loss(dist_a, dist_b, T, Na, Nb, reduction, frame_w, loss, s);
    return launched("chamfer_fwd launch");
}

}  // namespace dc

using namespace dc;

extern "C" {

int dc_version(void) { return 100; }

const char *dc_last_error(const dc_ctx *) { return g_err.c_str(); }

int dc_create(dc_ctx **out, int device, size_t hbm_budget_bytes, int max_slots) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return DC_ERR_INVALID;
    }
    *out = nullptr;
    int n = 0;
    DC_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) {
        set_error("device index out of range");
        return DC_ERR_INVALID;
    }
    if (max_slots < 0) {
        set_error("max_slots must be >= 0");
        return DC_ERR_INVALID;
    }
    DC_HIP(hipSetDevice(device));
    dc_ctx *c = new (std::nothrow) dc_ctx();
    if (!c) return DC_ERR_NOMEM;
    c->device = device;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t(64) << 30);
    c->max_slots = max_slots ? max_slots : 64;
    // the status and counter words are the first device memory held against the budget
    c->held = CTX_WORDS_BYTES;
    if (c->held > c->budget) {
        delete c;
        set_error("dc_create: the budget cannot hold the context's status words");
        return DC_ERR_BUDGET;
    }
    hipError_t e = hipMalloc(&c->d_status, sizeof(unsigned) * 4);
    if (e == hipSuccess) e = hipMalloc(&c->d_stats, STATS_BYTES);
    if (e == hipSuccess) e = hipMemset(c->d_status, 0, sizeof(unsigned) * 4);
    if (e == hipSuccess) e = hipMemset(c->d_stats, 0, STATS_BYTES);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->arena_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    const int rc = e == hipSuccess ? noalloc_init(device) : hip_fail(e, "dc_create");
    if (rc != DC_OK) {
        (void)hipFree(c->d_status);
        (void)hipFree(c->d_stats);
        if (c->arena_ev) (void)hipEventDestroy(c->arena_ev);
        delete c;
        return rc;
    }
    *out = c;
    return DC_OK;
}

int dc_destroy(dc_ctx *ctx) {
    clear_error();
    if (!ctx) return DC_ERR_INVALID;
    (void)hipSetDevice(ctx->device);
    if (ctx->sched) {
        sched_destroy(ctx);
        ctx->sched = nullptr;
    }
    (void)hipDeviceSynchronize();
    dev_free(ctx, ctx->arena.base, ctx->arena.cap);
    (void)hipFree(ctx->d_status);
    (void)hipFree(ctx->d_stats);
    (void)hipEventDestroy(ctx->arena_ev);
    delete ctx;
    return DC_OK;
}

int dc_sync(dc_ctx *ctx, void *stream) {
    clear_error();
    if (!ctx) return DC_ERR_INVALID;
    DC_HIP(hipSetDevice(ctx->device));
    DC_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    unsigned st = 0;
    DC_HIP(hipMemcpy(&st, ctx->d_status, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (st) DC_HIP(hipMemset(ctx->d_status, 0, sizeof(unsigned)));
    if (st & ST_BAD_FACE) {
        set_error("a face index lies outside [0, V)");
        return DC_ERR_INVALID;
    }
    if (st & ST_BAD_INDEX) {
        set_error("a body's vertex range lies outside [0, V] or is decreasing");
        return DC_ERR_INVALID;
    }
    if (st & ST_DEGENERATE) {
        set_error("a frame has zero or non-finite total surface area");
        return DC_ERR_DEGENERATE;
    }
    return DC_OK;
}

int dc_get_stats(dc_ctx *ctx, dc_stats *out) {
    clear_error();
    if (!ctx || !out) return DC_ERR_INVALID;
    DC_HIP(hipSetDevice(ctx->device));
    std::vector<unsigned long long> v((size_t)STATS_SLOTS * STATS_SLOT_WORDS);
    DC_HIP(hipMemcpy(v.data(), ctx->d_stats, STATS_BYTES, hipMemcpyDeviceToHost));
    out->queries = out->candidates = out->fallbacks = 0;
    for (int k = 0; k < STATS_SLOTS; ++k) {
        out->queries += v[(size_t)k * STATS_SLOT_WORDS];
        out->candidates += v[(size_t)k * STATS_SLOT_WORDS + 1];
        out->fallbacks += v[(size_t)k * STATS_SLOT_WORDS + 2];
    }
    return DC_OK;
}

int dc_profile(dc_ctx *ctx, int enable) {
    clear_error();
    if (!ctx) return DC_ERR_INVALID;
    ctx->prof = enable != 0;
    return DC_OK;
}

int dc_get_kernel_times(dc_ctx *ctx, dc_kernel_times *out, int reset) {
    clear_error();
    if (!ctx || !out) return DC_ERR_INVALID;
    DC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->prof_mu);
    for (auto &r : ctx->prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess &&
            hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            ctx->prof_ms[r.cat] += ms;
            ctx->prof_n[r.cat] += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ctx->prof_pending.clear();
    for (int k = 0; k < 4; ++k) {
        out->ms[k] = ctx->prof_ms[k];
        out->launches[k] = ctx->prof_n[k];
        if (reset) {
            ctx->prof_ms[k] = 0;
            ctx->prof_n[k] = 0;
        }
    }
    return DC_OK;
}

int dc_memory_held(dc_ctx *ctx, size_t *held, size_t *budget) {
    clear_error();
    if (!ctx || !held) return DC_ERR_INVALID;
    std::lock_guard<std::mutex> g(ctx->budget_mu);
    *held = ctx->held;
    if (budget) *budget = ctx->budget;
    return DC_OK;
}

int dc_debug_fail_allocs(dc_ctx *ctx, int n) {
    if (!ctx || n < 0) return DC_ERR_INVALID;
    std::lock_guard<std::mutex> g(ctx->budget_mu);
    ctx->fail_next_alloc = n;
    return DC_OK;
}

static int sample_surface_impl(dc_ctx *ctx, const float *verts, const int32_t *faces, int T,
                               int V, int F, int N, uint64_t seed, const uint32_t *uniforms,
                               const uint8_t *mask, int mask_per_frame, float *points,
                               int32_t *face_idx, float *bary, void *stream) {
    clear_error();
    if (!ctx || !verts || !faces || !points || !face_idx || !bary) {
        set_error("dc_sample_surface: NULL argument");
        return DC_ERR_INVALID;
    }
    int rc = check_dims(T, {V, F, N});
    if (rc) return rc;
    DC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->mu);
    rc = arena_reserve(ctx, sample_scratch_bytes(T, F), static_cast<hipStream_t>(stream));
    if (rc) return rc;
    ArenaUse use{ctx, static_cast<hipStream_t>(stream)};
    return enqueue_sample(ctx, verts, faces, T, V, F, N, seed, uniforms, mask, mask_per_frame,
                          points, face_idx, bary, ctx->arena, ctx->d_status,
                          static_cast<hipStream_t>(stream));
}

int dc_sample_surface(dc_ctx *ctx, const float *verts, const int32_t *faces, int T, int V, int F,
                      int N, uint64_t seed, const uint32_t *uniforms, float *points,
                      int32_t *face_idx, float *bary, void *stream) {
    return sample_surface_impl(ctx, verts, faces, T, V, F, N, seed, uniforms, nullptr, 0, points,
                               face_idx, bary, stream);
}

int dc_sample_surface_masked(dc_ctx *ctx, const float *verts, const int32_t *faces, int T, int V,
                             int F, int N, uint64_t seed, const uint32_t *uniforms,
                             const uint8_t *face_mask, int mask_per_frame, float *points,
                             int32_t *face_idx, float *bary, void *stream) {
    if (!face_mask || (mask_per_frame != 0 && mask_per_frame != 1)) {
        clear_error();
        set_error("dc_sample_surface_masked: NULL face_mask or mask_per_frame not 0/1");
        return DC_ERR_INVALID;
    }
    return sample_surface_impl(ctx, verts, faces, T, V, F, N, seed, uniforms, face_mask,
                               mask_per_frame, points, face_idx, bary, stream);
}

int dc_area_cdf(dc_ctx *ctx, const float *verts, const int32_t *faces, int T, int V, int F,
                const uint8_t *face_mask, int mask_per_frame, double *cdf, int32_t *last_face,
                void *stream) {
    clear_error();
    if (!ctx || !verts || !faces || !cdf || (mask_per_frame != 0 && mask_per_frame != 1)) {
        set_error("dc_area_cdf: NULL argument or mask_per_frame not 0/1");
        return DC_ERR_INVALID;
    }
    int rc = check_dims(T, {V, F});
    if (rc) return rc;
    DC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->mu);
    // the kernel always writes the last faces: to scratch when the caller does not want them
    rc = arena_reserve(ctx, sizeof(int32_t) * (size_t)T, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    ArenaUse use{ctx, static_cast<hipStream_t>(stream)};
    int32_t *lastpos = last_face ? last_face : ctx->arena.take<int32_t>((size_t)T);
    ProfScope ps(ctx, 2, static_cast<hipStream_t>(stream));
    launch_area_cdf(verts, faces, T, V, F, face_mask, face_mask ? mask_per_frame : 0, cdf,
                    lastpos, ctx->d_status, static_cast<hipStream_t>(stream));
    return launched("area_cdf launch");
}

int dc_sample_surface_bwd(dc_ctx *ctx, const float *grad_points, const int32_t *faces,
                          const int32_t *face_idx, const float *bary, int T, int V, int F, int N,
                          float *grad_verts, void *stream) {
    clear_error();
    if (!ctx || !grad_points || !faces || !face_idx || !bary || !grad_verts) {
        set_error("dc_sample_surface_bwd: NULL argument");
        return DC_ERR_INVALID;
    }
    int rc = check_dims(T, {V, F, N, 3L * F});
    if (rc) return rc;
    DC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->mu);
    const size_t need = sample_bwd_scratch_bytes(T, V, F, N);
    rc = arena_reserve(ctx, need, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    ArenaUse use{ctx, static_cast<hipStream_t>(stream)};
    ProfScope ps(ctx, 3, static_cast<hipStream_t>(stream));
    launch_sample_bwd(grad_points, faces, face_idx, bary, T, V, F, N, grad_verts,
                      ctx->arena.take<char>(need), static_cast<hipStream_t>(stream));
    return launched("sample_surface_bwd launch");
}

int dc_chamfer_fwd(dc_ctx *ctx, const float *a, const float *b, int T, int Na, int Nb,
                   int precision, int reduction, const float *frame_w, float *dist_a,
                   int32_t *idx_a, float *dist_b, int32_t *idx_b, double *loss, void *stream) {
    clear_error();
    if (!ctx || !a || !b || !dist_a || !idx_a || !loss) {
        set_error("dc_chamfer_fwd: NULL argument");
        return DC_ERR_INVALID;
    }
    if ((dist_b == nullptr) != (idx_b == nullptr) ||
        (!idx_b && reduction != DC_RED_SIM2REAL_SUM)) {
        set_error("dc_chamfer_fwd: dist_b and idx_b may be NULL (together) only for the "
                  "unidirectional reduction");
        return DC_ERR_INVALID;
    }
    if (precision != DC_PREC_FP32 && precision != DC_PREC_BF16_REFINE) {
        set_error("unknown precision");
        return DC_ERR_INVALID;
    }
    if (reduction != DC_RED_BIDIR_MEAN && reduction != DC_RED_SIM2REAL_SUM) {
        set_error("unknown reduction");
        return DC_ERR_INVALID;
    }
    int rc = check_dims(T, {Na, Nb});
    if (rc) return rc;
    DC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->mu);
    const size_t need = chamfer_fwd_scratch_bytes(T, Na, Nb, precision);
    rc = arena_reserve(ctx, need, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    ArenaUse use{ctx, static_cast<hipStream_t>(stream)};
    return enqueue_chamfer_fwd(ctx, a, b, T, Na, Nb, precision, reduction, frame_w, dist_a, idx_a,
                               dist_b, idx_b, loss, ctx->arena.take<char>(need), ctx->d_stats,
                               static_cast<hipStream_t>(stream));
}

int dc_chamfer_bwd(dc_ctx *ctx, const double *grad_loss, const float *a, const float *b,
                   const int32_t *idx_a, const int32_t *idx_b, int T, int Na, int Nb,
                   int reduction, const float *frame_w, float *grad_a, float *grad_b,
                   void *stream) {
    clear_error();
    if (!ctx || !grad_loss || !a || !b || !idx_a || !grad_a) {
        set_error("dc_chamfer_bwd: NULL argument");
        return DC_ERR_INVALID;
    }
    if (!idx_b && reduction != DC_RED_SIM2REAL_SUM) {
        set_error("dc_chamfer_bwd: idx_b may be NULL only for the unidirectional reduction");
        return DC_ERR_INVALID;
    }
    if (reduction != DC_RED_BIDIR_MEAN && reduction != DC_RED_SIM2REAL_SUM) {
        set_error("unknown reduction");
        return DC_ERR_INVALID;
    }
    int rc = check_dims(T, {Na, Nb});
    if (rc) return rc;
    DC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->mu);
    const size_t need = chamfer_bwd_scratch_bytes(T, Na, Nb, grad_b != nullptr);
    rc = arena_reserve(ctx, need, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    ArenaUse use{ctx, static_cast<hipStream_t>(stream)};
    ProfScope ps(ctx, 3, static_cast<hipStream_t>(stream));
    launch_chamfer_bwd(grad_loss, a, b, idx_a, idx_b, T, Na, Nb, reduction, frame_w, grad_a,
                       grad_b, ctx->arena.take<char>(need), static_cast<hipStream_t>(stream));
    return launched("chamfer_bwd launch");
}

int dc_rigid_pose(dc_ctx *ctx, const double *q, const float *p0, const int32_t *body_start,
                  int T, int B, int V, float *verts, void *stream) {
    clear_error();
    if (!ctx || !q || !p0 || !body_start || !verts) {
        set_error("dc_rigid_pose: NULL argument");
        return DC_ERR_INVALID;
    }
    int rc = check_dims(T, {B, V});
    if (rc) return rc;
    DC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->mu);
    launch_rigid_fwd(q, p0, body_start, T, B, V, verts, ctx->d_status,
                     static_cast<hipStream_t>(stream));
    return launched("rigid_pose launch");
}

int dc_rigid_pose_bwd(dc_ctx *ctx, const double *q, const float *p0, const int32_t *body_start,
                      const float *grad_verts, int T, int B, int V, double *grad_q,
                      void *stream) {
    clear_error();
    if (!ctx || !q || !p0 || !body_start || !grad_verts || !grad_q) {
        set_error("dc_rigid_pose_bwd: NULL argument");
        return DC_ERR_INVALID;
    }
    int rc = check_dims(T, {B, V});
    if (rc) return rc;
    DC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->mu);
    ProfScope ps(ctx, 3, static_cast<hipStream_t>(stream));
    launch_rigid_bwd(q, p0, body_start, grad_verts, T, B, V, grad_q, ctx->d_status,
                     static_cast<hipStream_t>(stream));
    return launched("rigid_pose_bwd launch");
}

int dc_submit(dc_ctx *ctx, const dc_request *req, dc_result *out, uint64_t *ticket) {
    clear_error();
    if (!ctx || !req || !out || !ticket) {
        set_error("dc_submit: NULL argument");
        return DC_ERR_INVALID;
    }
    return sched_submit(ctx, req, out, ticket);
}

int dc_request_bytes(const dc_request *req, int want_grad, size_t *bytes) {
    clear_error();
    if (!req || !bytes || req->T < 1 || req->V < 1 || req->F < 1 || req->n_sim < 1 ||
        req->n_obs < 1) {
        set_error("dc_request_bytes: invalid request");
        return DC_ERR_INVALID;
    }
    *bytes = request_bytes(req->T, req->V, req->F, req->n_sim, req->n_obs, req->precision,
                           want_grad != 0);
    return DC_OK;
}

int dc_poll(dc_ctx *ctx, uint64_t ticket) {
    clear_error();
    if (!ctx) return DC_ERR_INVALID;
    return sched_poll(ctx, ticket);
}

int dc_wait(dc_ctx *ctx, uint64_t ticket, int64_t timeout_us) {
    clear_error();
    if (!ctx) return DC_ERR_INVALID;
    return sched_wait(ctx, ticket, (long long)timeout_us);
}

}  // extern "C"
