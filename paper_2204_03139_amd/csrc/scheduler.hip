// Serving loop: continuous admission of calibration requests under an HBM budget.
//
// dc_submit copies a request's host inputs and queues it.  A scheduler thread admits queued
// requests in arrival order whenever a slot is free and the request's device footprint fits
// under the budget, uploads its inputs, and enqueues its whole pipeline (sampling, Chamfer
// forward, Chamfer backward, sampling backward, result download) on one of several streams, so
// requests admitted while others run overlap on the device.  Completion is detected with events;
// device memory then returns to the budget and dc_poll reports the result.  A request's work is
// enqueued with exactly the same launches as when it runs alone, so its results do not depend on
// what else is in flight.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "scheduler.h"

namespace dc {
namespace {

constexpr int NSTREAMS = 4;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

__global__ void k_fill_f64(double *p, int n, double v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(unsigned *p, int n, unsigned v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

enum { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct Req {
    uint64_t ticket = 0;
    dc_result *out = nullptr;
    int T = 0, V = 0, F = 0, Na = 0, Nb = 0, precision = 0, reduction = 0;
    uint64_t seed = 0;
    bool want_grad = false, has_w = false;
    std::vector<float> verts, obs, fw;
    std::vector<int32_t> faces;
    size_t bytes = 0;
    char *dmem = nullptr;
    int slot = -1;
    int stream = 0;
    hipEvent_t ev = nullptr;
    int state = Q_QUEUED;
    int status = DC_OK;
};

// pinned host staging for results, one per slot, grown on demand
struct Slot {
    char *host = nullptr;
    size_t cap = 0;
    bool busy = false;
};

}  // namespace

struct Scheduler {
    dc_ctx *ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;
    std::vector<Req *> running;
    std::unordered_map<uint64_t, Req *> table;
    std::vector<Slot> slots;
    uint64_t next_ticket = 1;
    bool stop = false;
    hipStream_t streams[NSTREAMS] = {};
    int rr = 0;
    std::thread th;
};

static size_t scratch_bytes(int T, int V, int F, int Na, int Nb, int precision, bool want_grad) {
    size_t s = sample_scratch_bytes(T, F);
    s = std::max(s, chamfer_fwd_scratch_bytes(T, Na, Nb, precision));
    if (want_grad) {
        s = std::max(s, chamfer_bwd_scratch_bytes(T, Na, Nb, false));
        s = std::max(s, sample_bwd_scratch_bytes(T, V, F, Na));
    }
    return s;
}

size_t request_bytes(int T, int V, int F, int Na, int Nb, int precision, bool want_grad) {
    const size_t TV = (size_t)T * V, TA = (size_t)T * Na, TB = (size_t)T * Nb;
    size_t b = 0;
    b += Arena::need(TV * 3, 4) + Arena::need((size_t)F * 3, 4) + Arena::need(TB * 3, 4);
    b += Arena::need(T, 4) + Arena::need(4, 4);                         // frame weights, status
    b += Arena::need(TA * 3, 4) * 2 + Arena::need(TA, 4);              // points, bary, face_idx
    b += Arena::need(TA, 4) * 2 + Arena::need(TB, 4) * 2 + Arena::need(T, 8);  // nn + loss
    if (want_grad)
        b += Arena::need(T, 8) + Arena::need(TA * 3, 4) + Arena::need(TV * 3, 4);
    b += scratch_bytes(T, V, F, Na, Nb, precision, want_grad);
    return b;
}

static size_t host_bytes(const Req *r) {
    return Arena::need((size_t)r->T, 8) + Arena::need(16, 1) +
           (r->want_grad ? Arena::need((size_t)r->T * r->V * 3, 4) : 0);
}

// enqueue the request's whole pipeline on its stream; returns a status code
static int run_request(Scheduler *S, Req *r) {
    dc_ctx *ctx = S->ctx;
    hipStream_t s = S->streams[r->stream];
    {
        std::lock_guard<std::mutex> g(ctx->budget_mu);
        if (ctx->fail_next_alloc > 0) {  // test hook: a forced allocation failure
            --ctx->fail_next_alloc;
            set_error("device allocation failed (forced)");
            return DC_ERR_NOMEM;
        }
    }
    if (hipMallocAsync(reinterpret_cast<void **>(&r->dmem), r->bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        r->dmem = nullptr;
        set_error("device allocation of a request failed");
        return DC_ERR_NOMEM;
    }
    Arena ar;
    ar.base = r->dmem;
    ar.cap = r->bytes;
    const int T = r->T, V = r->V, F = r->F, Na = r->Na, Nb = r->Nb;
    const size_t TV = (size_t)T * V, TA = (size_t)T * Na, TB = (size_t)T * Nb;
    float *verts = ar.take<float>(TV * 3);
    int32_t *faces = ar.take<int32_t>((size_t)F * 3);
    float *obs = ar.take<float>(TB * 3);
    float *fw = ar.take<float>(T);
    unsigned *status = ar.take<unsigned>(4);
    float *pts = ar.take<float>(TA * 3);
    float *bary = ar.take<float>(TA * 3);
    int32_t *fidx = ar.take<int32_t>(TA);
    float *da = ar.take<float>(TA);
    int32_t *ia = ar.take<int32_t>(TA);
    float *db = ar.take<float>(TB);
    int32_t *ib = ar.take<int32_t>(TB);
    double *loss = ar.take<double>(T);
    double *gl = nullptr;
    float *gpts = nullptr, *gverts = nullptr;
    if (r->want_grad) {
        gl = ar.take<double>(T);
        gpts = ar.take<float>(TA * 3);
        gverts = ar.take<float>(TV * 3);
    }
    char *scratch = ar.take<char>(scratch_bytes(T, V, F, Na, Nb, r->precision, r->want_grad));

    DC_HIP(hipMemcpyAsync(verts, r->verts.data(), TV * 3 * 4, hipMemcpyHostToDevice, s));
    DC_HIP(hipMemcpyAsync(faces, r->faces.data(), (size_t)F * 3 * 4, hipMemcpyHostToDevice, s));
    DC_HIP(hipMemcpyAsync(obs, r->obs.data(), TB * 3 * 4, hipMemcpyHostToDevice, s));
    if (r->has_w) DC_HIP(hipMemcpyAsync(fw, r->fw.data(), (size_t)T * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, status, 4, 0u);

    Arena sar;
    sar.base = scratch;
    sar.cap = r->bytes;
    int rc = enqueue_sample(nullptr, verts, faces, T, V, F, Na, r->seed, nullptr, pts, fidx, bary, sar,
                            status, s);
    if (rc) return rc;
    rc = enqueue_chamfer_fwd(nullptr, pts, obs, T, Na, Nb, r->precision, r->reduction,
                             r->has_w ? fw : nullptr, da, ia, db, ib, loss, scratch, ctx->d_stats,
                             s);
    if (rc) return rc;
    if (r->want_grad) {
        hipLaunchKernelGGL(k_fill_f64, dim3((T + 255) / 256), dim3(256), 0, s, gl, T, 1.0);
        launch_chamfer_bwd(gl, pts, obs, ia, ib, T, Na, Nb,
                           r->reduction, r->has_w ? fw : nullptr, gpts, nullptr, scratch, s);
        launch_sample_bwd(gpts, faces, fidx, bary, T, V, F, Na, gverts, scratch, s);
    }
    Slot &sl = S->slots[r->slot];
    char *h = sl.host;
    DC_HIP(hipMemcpyAsync(h, loss, (size_t)T * 8, hipMemcpyDeviceToHost, s));
    DC_HIP(hipMemcpyAsync(h + Arena::need(T, 8), status, 16, hipMemcpyDeviceToHost, s));
    if (r->want_grad)
        DC_HIP(hipMemcpyAsync(h + Arena::need(T, 8) + Arena::need(16, 1), gverts, TV * 3 * 4,
                              hipMemcpyDeviceToHost, s));
    DC_HIP(hipFreeAsync(r->dmem, s));
    r->dmem = nullptr;
    DC_HIP(hipEventRecord(r->ev, s));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "serving launch");
    return DC_OK;
}

static void finish(Scheduler *S, Req *r) {
    if (r->status == DC_OK) {
        const char *h = S->slots[r->slot].host;
        std::memcpy(r->out->loss, h, (size_t)r->T * 8);
        unsigned st = 0;
        std::memcpy(&st, h + Arena::need(r->T, 8), 4);
        if (st & ST_BAD_FACE)
            r->status = DC_ERR_INVALID;
        else if (st & ST_DEGENERATE)
            r->status = DC_ERR_DEGENERATE;
        if (r->want_grad)
            std::memcpy(r->out->grad_verts, h + Arena::need(r->T, 8) + Arena::need(16, 1),
                        (size_t)r->T * r->V * 3 * 4);
    }
    if (r->slot >= 0) S->slots[r->slot].busy = false;
    budget_give(S->ctx, r->bytes);
    r->out->t_done = now_s();
    r->out->status = r->status;
    r->state = Q_DONE;
    // free the input copies now; the record itself lives until polled
    std::vector<float>().swap(r->verts);
    std::vector<float>().swap(r->obs);
    std::vector<int32_t>().swap(r->faces);
}

static void loop(Scheduler *S) {
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        if (S->stop && S->queue.empty() && S->running.empty()) break;
        // admit in arrival order while a slot and the budget allow
        while (!S->queue.empty() && (int)S->running.size() < S->ctx->max_slots) {
            Req *r = S->queue.front();
            if (budget_take(S->ctx, r->bytes) != DC_OK) break;
            S->queue.pop_front();
            int slot = -1;
            for (size_t k = 0; k < S->slots.size(); ++k)
                if (!S->slots[k].busy) {
                    slot = (int)k;
                    break;
                }
            Slot &sl = S->slots[slot];
            sl.busy = true;
            r->slot = slot;
            r->stream = S->rr;
            S->rr = (S->rr + 1) % NSTREAMS;
            r->state = Q_RUNNING;
            r->out->t_admit = now_s();
            const size_t hb = host_bytes(r);
            int rc = DC_OK;
            if (sl.cap < hb) {
                if (sl.host) (void)hipHostFree(sl.host);
                sl.host = nullptr;
                sl.cap = 0;
                if (hipHostMalloc(reinterpret_cast<void **>(&sl.host), hb, 0) != hipSuccess) {
                    sl.host = nullptr;
                    rc = DC_ERR_NOMEM;
                } else {
                    sl.cap = hb;
                }
            }
            if (rc == DC_OK && hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess)
                rc = DC_ERR_HIP;
            if (rc == DC_OK) rc = run_request(S, r);
            S->running.push_back(r);
            if (rc != DC_OK) {
                r->status = rc;
                // wait for anything already enqueued for it before releasing its memory
                (void)hipStreamSynchronize(S->streams[r->stream]);
                if (r->dmem) (void)hipFree(r->dmem);
                r->dmem = nullptr;
            }
        }
        bool progressed = false;
        for (size_t k = 0; k < S->running.size();) {
            Req *r = S->running[k];
            bool done = r->status != DC_OK;
            if (!done && hipEventQuery(r->ev) == hipSuccess) done = true;
            if (done) {
                if (r->ev) (void)hipEventDestroy(r->ev);
                r->ev = nullptr;
                finish(S, r);
                S->running.erase(S->running.begin() + k);
                progressed = true;
            } else {
                ++k;
            }
        }
        if (!progressed) S->cv.wait_for(lk, std::chrono::microseconds(50));
    }
}

static int ensure_scheduler(dc_ctx *ctx) {
    if (ctx->sched) return DC_OK;
    Scheduler *S = new Scheduler();
    S->ctx = ctx;
    S->slots.resize(ctx->max_slots);
    DC_HIP(hipSetDevice(ctx->device));
    for (int k = 0; k < NSTREAMS; ++k)
        DC_HIP(hipStreamCreateWithFlags(&S->streams[k], hipStreamNonBlocking));
    S->th = std::thread(loop, S);
    ctx->sched = S;
    return DC_OK;
}

int sched_submit(dc_ctx *ctx, const dc_request *q, dc_result *out, uint64_t *ticket) {
    if (!q->verts || !q->faces || !q->observed || !out->loss) {
        set_error("dc_submit: NULL input or loss buffer");
        return DC_ERR_INVALID;
    }
    if (q->T < 1 || q->T > 65535 || q->V < 1 || q->F < 1 || q->n_sim < 1 || q->n_obs < 1 ||
        q->V > (1 << 24) || q->F > (1 << 24) || q->n_sim > (1 << 24) || q->n_obs > (1 << 24)) {
        set_error("dc_submit: size out of range");
        return DC_ERR_INVALID;
    }
    if ((q->precision != DC_PREC_FP32 && q->precision != DC_PREC_BF16_REFINE) ||
        (q->reduction != DC_RED_BIDIR_MEAN && q->reduction != DC_RED_SIM2REAL_SUM)) {
        set_error("dc_submit: unknown precision or reduction");
        return DC_ERR_INVALID;
    }
    const bool want_grad = out->grad_verts != nullptr;
    const size_t bytes =
        request_bytes(q->T, q->V, q->F, q->n_sim, q->n_obs, q->precision, want_grad);
    if (bytes > ctx->budget) {
        set_error("dc_submit: request needs " + std::to_string(bytes) +
                  " bytes, more than the whole budget");
        return DC_ERR_BUDGET;
    }
    Req *r = new Req();
    r->out = out;
    r->T = q->T;
    r->V = q->V;
    r->F = q->F;
    r->Na = q->n_sim;
    r->Nb = q->n_obs;
    r->precision = q->precision;
    r->reduction = q->reduction;
    r->seed = q->seed;
    r->want_grad = want_grad;
    r->bytes = bytes;
    r->verts.assign(q->verts, q->verts + (size_t)q->T * q->V * 3);
    r->faces.assign(q->faces, q->faces + (size_t)q->F * 3);
    r->obs.assign(q->observed, q->observed + (size_t)q->T * q->n_obs * 3);
    if (q->frame_w) {
        r->has_w = true;
        r->fw.assign(q->frame_w, q->frame_w + q->T);
    }
    out->t_submit = now_s();
    out->t_admit = 0;
    out->t_done = 0;
    out->status = DC_PENDING;
    std::lock_guard<std::mutex> g(ctx->mu);  // creation of the loop is serialised with direct calls
    int rc = ensure_scheduler(ctx);
    if (rc) {
        delete r;
        return rc;
    }
    Scheduler *S = ctx->sched;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next_ticket++;
        S->table[r->ticket] = r;
        S->queue.push_back(r);
        *ticket = r->ticket;
    }
    S->cv.notify_one();
    return DC_OK;
}

int sched_poll(dc_ctx *ctx, uint64_t ticket) {
    Scheduler *S = ctx->sched;
    if (!S) {
        set_error("dc_poll: unknown ticket");
        return DC_ERR_INVALID;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->table.find(ticket);
    if (it == S->table.end()) {
        set_error("dc_poll: unknown ticket");
        return DC_ERR_INVALID;
    }
    Req *r = it->second;
    if (r->state != Q_DONE) return DC_PENDING;
    const int st = r->status;
    S->table.erase(it);
    delete r;
    return st;
}

void sched_destroy(dc_ctx *ctx) {
    Scheduler *S = ctx->sched;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_one();
    S->th.join();
    for (auto &kv : S->table) delete kv.second;
    for (auto &sl : S->slots)
        if (sl.host) (void)hipHostFree(sl.host);
    for (int k = 0; k < NSTREAMS; ++k)
        if (S->streams[k]) (void)hipStreamDestroy(S->streams[k]);
    delete S;
}

}  // namespace dc
