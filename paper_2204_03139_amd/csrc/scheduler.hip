// Serving loop: continuous batching of calibration requests under an HBM budget, replayed as
// captured graphs of persistent kernels.
//
// dc_submit copies a request's host inputs and queues it.  A scheduler thread forms batches from
// the queue in arrival order (at most MAX_BATCH requests, a bounded amount of pair work, the
// context's slot limit and its HBM budget), and runs each batch on one of NSLOTS batch slots, so
// requests that arrive while others are on the device are admitted into the next free slot and
// their work overlaps with the batches already running.
//
// A batch runs as one replay of a graph built once per slot: the fixed program below, one
// persistent kernel node per stage, with the stages that have no work in the batch switched off.
// For every request the host code of the direct calls is run in recording mode, which yields the
// request's launches (kernel, logical grid, parameters) instead of executing them; each launch is
// assigned, in order, to the next program stage of its kernel, and the batch's stage tables are
// uploaded to the slot's device descriptor before the replay.
// Inputs are uploaded from pinned staging in one copy per request, results come back the same
// way, and an event marks the batch's completion.  Every request executes exactly the launches
// of its direct calls, so its results do not depend on what it is batched with.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"
#include "scheduler.h"

namespace dc {
namespace {

constexpr int NSLOTS = 3;              // batches in flight
constexpr double BATCH_PAIRS = 5e9;    // pair work that closes a batch (about 0.5 ms of device time)
constexpr int FILL_THREADS = 256;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct FillU32Params {
    unsigned *p;
    int n;
    unsigned v;
};

struct FillF64Params {
    double *p;
    double v;
    int n;
    int pad;
};

__device__ __forceinline__ void fill_u32_body(const FillU32Params &q, const Blk &b) {
    const int i = b.x * FILL_THREADS + threadIdx.x;
    if (i < q.n) q.p[i] = q.v;
}

__device__ __forceinline__ void fill_f64_body(const FillF64Params &q, const Blk &b) {
    const int i = b.x * FILL_THREADS + threadIdx.x;
    if (i < q.n) q.p[i] = q.v;
}

__global__ __launch_bounds__(FILL_THREADS) void k_fill_u32(FillU32Params q) {
    fill_u32_body(q, grid_blk());
}

__global__ __launch_bounds__(FILL_THREADS) void k_fill_f64(FillF64Params q) {
    fill_f64_body(q, grid_blk());
}

void fill_u32(unsigned *p, int n, unsigned v, hipStream_t s) {
    FillU32Params q;
    q.p = p;
    q.n = n;
    q.v = v;
    dispatch(KT_FILL_U32, k_fill_u32, dim3((n + FILL_THREADS - 1) / FILL_THREADS), FILL_THREADS, q,
             s);
}

void fill_f64(double *p, int n, double v, hipStream_t s) {
    FillF64Params q;
    q.p = p;
    q.v = v;
    q.n = n;
    q.pad = 0;
    dispatch(KT_FILL_F64, k_fill_f64, dim3((n + FILL_THREADS - 1) / FILL_THREADS), FILL_THREADS, q,
             s);
}

// The serving program: every request's recorded launches form a subsequence of it.  Exact
// searches may use any of the three queries-per-lane variants; each sort has room for four
// 8-bit digit passes (keys below 2^32).
#define SORT_PASSES                                                                           \
    KT_SS_HIST, KT_SS_SCAN, KT_SS_SCATTER, KT_SS_HIST, KT_SS_SCAN, KT_SS_SCATTER, KT_SS_HIST, \
        KT_SS_SCAN, KT_SS_SCATTER, KT_SS_HIST, KT_SS_SCAN, KT_SS_SCATTER
const int PROGRAM[] = {
    KT_FILL_U32,  KT_AREA_CDF, KT_SAMPLE,                                      // sampling
    KT_NORM_MAX,  KT_NORM_MAX, KT_PACK,     KT_SCREEN, KT_SCREEN_ROWS, KT_REFINE,  // screen
    KT_NN8,       KT_NN4,      KT_NN1,      KT_NN_MERGE,   // exact a -> b (or its heavy rows)
    KT_COLMERGE,  KT_COLREFINE,                            // screen, columns
    KT_NN8,       KT_NN4,      KT_NN1,      KT_NN_MERGE,   // exact b -> a (or its heavy columns)
    KT_LOSS,      KT_FILL_F64, SORT_PASSES, KT_CHAMFER_BWD,                    // Chamfer bwd
    SORT_PASSES,  KT_BOUNDS,   SORT_PASSES, KT_BOUNDS,  KT_FACE_GRAD, KT_VERTEX_GRAD};
#undef SORT_PASSES
constexpr int NPROG = (int)(sizeof(PROGRAM) / sizeof(PROGRAM[0]));
static_assert(NPROG <= MAX_STAGES, "program longer than the descriptor");

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
    double pairs = 0;
    int state = Q_QUEUED;
    int status = DC_OK;
    // within the batch
    size_t dev_off = 0, in_off = 0, out_off = 0;
    std::vector<OpRec> ops;
    std::vector<int> stage_of;
};

// device pieces of one request, carved from its region: inputs, then outputs, then the rest
struct Layout {
    float *verts, *obs, *fw, *pts, *bary, *da, *db, *gpts, *gverts;
    int32_t *faces, *fidx, *ia, *ib;
    double *loss, *gl;
    unsigned *status;
    char *scratch;
    size_t in_bytes, out_bytes;
};

size_t scratch_bytes(int T, int V, int F, int Na, int Nb, int precision, bool want_grad) {
    size_t s = sample_scratch_bytes(T, F);
    s = std::max(s, chamfer_fwd_scratch_bytes(T, Na, Nb, precision));
    if (want_grad) {
        s = std::max(s, chamfer_bwd_scratch_bytes(T, Na, Nb, false));
        s = std::max(s, sample_bwd_scratch_bytes(T, V, F, Na));
    }
    return s;
}

Layout carve(const Req *r, char *base) {
    Arena ar;
    ar.base = base;
    ar.cap = r->bytes;
    const int T = r->T, V = r->V, F = r->F, Na = r->Na, Nb = r->Nb;
    const size_t TV = (size_t)T * V, TA = (size_t)T * Na, TB = (size_t)T * Nb;
    Layout L;
    L.verts = ar.take<float>(TV * 3);
    L.faces = ar.take<int32_t>((size_t)F * 3);
    L.obs = ar.take<float>(TB * 3);
    L.fw = ar.take<float>(T);
    L.in_bytes = ar.off;
    L.loss = ar.take<double>(T);
    L.status = ar.take<unsigned>(4);
    L.gverts = r->want_grad ? ar.take<float>(TV * 3) : nullptr;
    L.out_bytes = ar.off - L.in_bytes;
    L.pts = ar.take<float>(TA * 3);
    L.bary = ar.take<float>(TA * 3);
    L.fidx = ar.take<int32_t>(TA);
    L.da = ar.take<float>(TA);
    L.ia = ar.take<int32_t>(TA);
    L.db = ar.take<float>(TB);
    L.ib = ar.take<int32_t>(TB);
    L.gl = r->want_grad ? ar.take<double>(T) : nullptr;
    L.gpts = r->want_grad ? ar.take<float>(TA * 3) : nullptr;
    L.scratch = ar.take<char>(scratch_bytes(T, V, F, Na, Nb, r->precision, r->want_grad));
    return L;
}

// the launches of a request's whole pipeline, issued through dispatch()
int issue_request(const Req *r, const Layout &L, unsigned long long *stats) {
    const int T = r->T, V = r->V, F = r->F, Na = r->Na, Nb = r->Nb;
    hipStream_t s = nullptr;  // unused while recording
    fill_u32(L.status, 4, 0u, s);
    Arena sar;
    sar.base = L.scratch;
    sar.cap = r->bytes;
    int rc = enqueue_sample(nullptr, L.verts, L.faces, T, V, F, Na, r->seed, nullptr, nullptr, 0,
                            L.pts, L.fidx, L.bary, sar, L.status, s);
    if (rc) return rc;
    // the unidirectional loss needs neither the b -> a search nor its indices
    const bool cols = r->reduction != DC_RED_SIM2REAL_SUM;
    rc = enqueue_chamfer_fwd(nullptr, L.pts, L.obs, T, Na, Nb, r->precision, r->reduction,
                             r->has_w ? L.fw : nullptr, L.da, L.ia, cols ? L.db : nullptr,
                             cols ? L.ib : nullptr, L.loss, L.scratch, stats, s);
    if (rc) return rc;
    if (r->want_grad) {
        fill_f64(L.gl, T, 1.0, s);
        launch_chamfer_bwd(L.gl, L.pts, L.obs, L.ia, cols ? L.ib : nullptr, T, Na, Nb, r->reduction,
                           r->has_w ? L.fw : nullptr, L.gpts, nullptr, L.scratch, s);
        launch_sample_bwd(L.gpts, L.faces, L.fidx, L.bary, T, V, F, Na, L.gverts, L.scratch, s);
    }
    return DC_OK;
}

// record a request's launches against a region at `base` and assign them to program stages
int plan_request(Req *r, char *base, unsigned long long *stats) {
    Recording rec;
    g_record = &rec;
    const Layout L = carve(r, base);
    const int rc = issue_request(r, L, stats);
    g_record = nullptr;
    if (rc) return rc;
    r->ops.swap(rec.ops);
    r->stage_of.assign(r->ops.size(), -1);
    int pos = 0;
    for (size_t k = 0; k < r->ops.size(); ++k) {
        while (pos < NPROG && PROGRAM[pos] != rec.types[k]) ++pos;
        const long items = (long)r->ops[k].gx * r->ops[k].gy * r->ops[k].gz;
        if (pos == NPROG || items > (1L << 26)) {
            set_error("request does not fit the serving program");
            return DC_ERR_UNSUPPORTED;
        }
        r->stage_of[k] = pos++;
    }
    return DC_OK;
}

// one batch slot: a stream, the captured program over the slot's descriptor, pinned staging
struct BatchSlot {
    hipStream_t stream = nullptr;
    BatchDesc *d_desc = nullptr;
    BatchDesc *h_desc = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t nodes[MAX_STAGES] = {};
    bool enabled[MAX_STAGES] = {};
    char *h_in = nullptr, *h_out = nullptr;
    size_t in_cap = 0, out_cap = 0;
    // the batch's device region: owned by the slot and grown when a batch needs more (a
    // per-batch stream-ordered allocation and free cost 0.35 ms of host time per batch)
    char *dmem = nullptr;
    size_t dcap = 0;
    hipEvent_t ev = nullptr;
    std::vector<Req *> reqs;
    bool busy = false;
};

int grow_pinned(char **p, size_t *cap, size_t need) {
    if (*cap >= need) return DC_OK;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t n = std::max(need, (size_t)1 << 20) * 5 / 4;
    if (hipHostMalloc(reinterpret_cast<void **>(p), n, 0) != hipSuccess) {
        *p = nullptr;
        set_error("pinned staging allocation failed");
        return DC_ERR_NOMEM;
    }
    *cap = n;
    return DC_OK;
}

}  // namespace

struct Scheduler {
    dc_ctx *ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;
    std::unordered_map<uint64_t, Req *> table;
    uint64_t next_ticket = 1;
    int running = 0;  // requests admitted and not finished
    bool stop = false;
    BatchedKernel kern[KT_COUNT] = {};
    BatchSlot slots[NSLOTS];
    std::thread th;
};

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

static void finish_req(Scheduler *S, Req *r, const char *h) {
    if (r->status == DC_OK && h) {
        std::memcpy(r->out->loss, h, (size_t)r->T * 8);
        unsigned st = 0;
        std::memcpy(&st, h + Arena::need(r->T, 8), 4);
        if (st & ST_BAD_FACE)
            r->status = DC_ERR_INVALID;
        else if (st & ST_DEGENERATE)
            r->status = DC_ERR_DEGENERATE;
        if (r->want_grad)
            std::memcpy(r->out->grad_verts, h + Arena::need(r->T, 8) + Arena::need(4, 4),
                        (size_t)r->T * r->V * 3 * 4);
    }
    budget_give(S->ctx, r->bytes);
    --S->running;
    r->out->t_done = now_s();
    r->out->status = r->status;
    r->state = Q_DONE;
    std::vector<float>().swap(r->verts);
    std::vector<float>().swap(r->obs);
    std::vector<int32_t>().swap(r->faces);
    std::vector<OpRec>().swap(r->ops);
}

// upload, replay and download one batch on slot `sl`; on failure every request of the batch
// fails with the returned status
static int run_batch(Scheduler *S, BatchSlot &sl) {
    hipStream_t s = sl.stream;
    size_t dbytes = 0, in_bytes = 0, out_bytes = 0;
    for (Req *r : sl.reqs) {
        r->dev_off = dbytes;
        dbytes += Arena::need(r->bytes, 1);
    }
    if (dbytes > sl.dcap) {  // the slot is idle: its previous batch no longer uses the region
        if (sl.dmem) (void)hipFree(sl.dmem);
        sl.dmem = nullptr;
        sl.dcap = 0;
        const size_t want = dbytes + dbytes / 4;
        if (hipMalloc(reinterpret_cast<void **>(&sl.dmem), want) != hipSuccess) {
            (void)hipGetLastError();
            sl.dmem = nullptr;
            set_error("device allocation of a batch failed");
            return DC_ERR_NOMEM;
        }
        sl.dcap = want;
    }
    // record every request against its region, then lay the stages out
    std::vector<Layout> lay;
    for (Req *r : sl.reqs) {
        const int rc = plan_request(r, sl.dmem + r->dev_off, S->ctx->d_stats);
        if (rc) return rc;
        lay.push_back(carve(r, sl.dmem + r->dev_off));
        r->in_off = in_bytes;
        r->out_off = out_bytes;
        in_bytes += lay.back().in_bytes;
        out_bytes += lay.back().out_bytes;
    }
    int rc = grow_pinned(&sl.h_in, &sl.in_cap, in_bytes);
    if (rc == DC_OK) rc = grow_pinned(&sl.h_out, &sl.out_cap, out_bytes);
    if (rc) return rc;
    BatchDesc *D = sl.h_desc;
    int nops = 0;
    for (int st = 0; st < NPROG; ++st) {
        D->stage[st].first = nops;
        D->stage[st].nops = 0;
        long total = 0;
        for (Req *r : sl.reqs)
            for (size_t k = 0; k < r->ops.size(); ++k) {
                if (r->stage_of[k] != st) continue;
                OpRec &o = D->op[nops++];
                o = r->ops[k];
                o.start = (int)total;
                total += (long)o.gx * o.gy * o.gz;
                ++D->stage[st].nops;
            }
        D->stage[st].total = (int)total;
    }
    // inputs: one copy per request from pinned staging laid out like its device region
    for (size_t q = 0; q < sl.reqs.size(); ++q) {
        const Req *r = sl.reqs[q];
        const Layout &L = lay[q];
        char *h = sl.h_in + r->in_off;
        const char *d0 = reinterpret_cast<const char *>(L.verts);
        std::memcpy(h, r->verts.data(), r->verts.size() * 4);
        std::memcpy(h + (reinterpret_cast<const char *>(L.faces) - d0), r->faces.data(),
                    r->faces.size() * 4);
        std::memcpy(h + (reinterpret_cast<const char *>(L.obs) - d0), r->obs.data(),
                    r->obs.size() * 4);
        if (r->has_w)
            std::memcpy(h + (reinterpret_cast<const char *>(L.fw) - d0), r->fw.data(),
                        r->fw.size() * 4);
        DC_HIP(hipMemcpyAsync(L.verts, h, L.in_bytes, hipMemcpyHostToDevice, s));
    }
    const size_t dsz = sizeof(D->stage) + (size_t)nops * sizeof(OpRec);
    DC_HIP(hipMemcpyAsync(sl.d_desc, D, dsz, hipMemcpyHostToDevice, s));
    // stages without work in this batch are switched off (the slot is idle, so its executable
    // graph may be updated)
    for (int st = 0; st < NPROG; ++st) {
        const bool on = D->stage[st].total > 0;
        if (on != sl.enabled[st]) {
            DC_HIP(hipGraphNodeSetEnabled(sl.exec, sl.nodes[st], on ? 1u : 0u));
            sl.enabled[st] = on;
        }
    }
    DC_HIP(hipGraphLaunch(sl.exec, s));
    for (size_t q = 0; q < sl.reqs.size(); ++q) {
        const Layout &L = lay[q];
        DC_HIP(hipMemcpyAsync(sl.h_out + sl.reqs[q]->out_off, L.loss, L.out_bytes,
                              hipMemcpyDeviceToHost, s));
    }
    DC_HIP(hipEventRecord(sl.ev, s));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "serving batch launch");
    return DC_OK;
}

static void fail_batch(Scheduler *S, BatchSlot &sl, int rc) {
    (void)hipStreamSynchronize(sl.stream);  // anything already enqueued has finished
    for (Req *r : sl.reqs) {
        r->status = rc;
        finish_req(S, r, nullptr);
    }
    sl.reqs.clear();
    sl.busy = false;
}

// take queued requests for a new batch in arrival order; false when nothing can be admitted
static bool form_batch(Scheduler *S, BatchSlot &sl) {
    double pairs = 0;
    while (!S->queue.empty() && (int)sl.reqs.size() < MAX_BATCH &&
           S->running < S->ctx->max_slots) {
        Req *r = S->queue.front();
        if (!sl.reqs.empty() && pairs + r->pairs > BATCH_PAIRS) break;
        if (budget_take(S->ctx, r->bytes) != DC_OK) break;
        S->queue.pop_front();
        ++S->running;
        r->state = Q_RUNNING;
        r->out->t_admit = now_s();
        bool fail = false;
        {
            std::lock_guard<std::mutex> g(S->ctx->budget_mu);
            if (S->ctx->fail_next_alloc > 0) {  // test hook: a forced allocation failure
                --S->ctx->fail_next_alloc;
                fail = true;
            }
        }
        if (fail) {
            r->status = DC_ERR_NOMEM;
            finish_req(S, r, nullptr);
            continue;
        }
        sl.reqs.push_back(r);
        pairs += r->pairs;
    }
    return !sl.reqs.empty();
}

static void loop(Scheduler *S) {
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool any_busy = false;
        for (auto &sl : S->slots) any_busy |= sl.busy;
        if (S->stop && S->queue.empty() && !any_busy) break;
        bool progressed = false;
        for (auto &sl : S->slots) {
            if (sl.busy) continue;
            if (!form_batch(S, sl)) {
                if (S->queue.empty()) break;
                continue;
            }
            sl.busy = true;
            progressed = true;
            // staging and launching run unlocked: the slot and its requests belong to this
            // thread until they finish, and submit / poll only touch the queue and the table
            lk.unlock();
            const int rc = run_batch(S, sl);
            lk.lock();
            if (rc != DC_OK) fail_batch(S, sl, rc);
        }
        for (auto &sl : S->slots) {
            if (!sl.busy || hipEventQuery(sl.ev) != hipSuccess) continue;
            for (Req *r : sl.reqs) finish_req(S, r, sl.h_out + r->out_off);
            sl.reqs.clear();
            sl.busy = false;
            progressed = true;
        }
        if (!progressed) S->cv.wait_for(lk, std::chrono::microseconds(50));
    }
}

static int init_slot(Scheduler *S, BatchSlot &sl) {
    DC_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    DC_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    DC_HIP(hipMalloc(reinterpret_cast<void **>(&sl.d_desc), sizeof(BatchDesc)));
    DC_HIP(hipHostMalloc(reinterpret_cast<void **>(&sl.h_desc), sizeof(BatchDesc), 0));
    // an empty descriptor: a replay before the first upload does nothing
    std::memset(sl.h_desc, 0, sizeof(BatchDesc));
    DC_HIP(hipMemcpy(sl.d_desc, sl.h_desc, sizeof(sl.h_desc->stage), hipMemcpyHostToDevice));
    // the program as a chain of kernel nodes over the slot's descriptor
    DC_HIP(hipGraphCreate(&sl.graph, 0));
    for (int st = 0; st < NPROG; ++st) {
        const BatchedKernel &k = S->kern[PROGRAM[st]];
        const BatchDesc *desc = sl.d_desc;
        int stage = st;
        void *args[2] = {&desc, &stage};
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof(kp));
        kp.func = const_cast<void *>(k.func);
        kp.gridDim = dim3(k.blocks);
        kp.blockDim = dim3(k.threads);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        DC_HIP(hipGraphAddKernelNode(&sl.nodes[st], sl.graph, st ? &sl.nodes[st - 1] : nullptr,
                                     st ? 1 : 0, &kp));
        sl.enabled[st] = true;
    }
    DC_HIP(hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0));
    return DC_OK;
}

static void release_slot(BatchSlot &sl) {
    if (sl.dmem) (void)hipFree(sl.dmem);
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    if (sl.graph) (void)hipGraphDestroy(sl.graph);
    if (sl.d_desc) (void)hipFree(sl.d_desc);
    if (sl.h_desc) (void)hipHostFree(sl.h_desc);
    if (sl.h_in) (void)hipHostFree(sl.h_in);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
}

static int ensure_scheduler(dc_ctx *ctx) {
    if (ctx->sched) return DC_OK;
    Scheduler *S = new Scheduler();
    S->ctx = ctx;
    register_sample_kernels(S->kern);
    register_nn_kernels(S->kern);
    register_screen_kernels(S->kern);
    register_sort_kernels(S->kern);
    register_backward_kernels(S->kern);
    register_fill_kernels(S->kern);
    for (int k = 0; k < KT_COUNT; ++k)
        if (!S->kern[k].func) {
            delete S;
            set_error("serving program: a kernel has no batched form");
            return DC_ERR_HIP;
        }
    int rc = DC_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) rc = DC_ERR_HIP;
    for (auto &sl : S->slots)
        if (rc == DC_OK) rc = init_slot(S, sl);
    if (rc != DC_OK) {
        for (auto &sl : S->slots) release_slot(sl);
        delete S;
        return rc;
    }
    S->th = std::thread(loop, S);
    ctx->sched = S;
    return DC_OK;
}

void register_fill_kernels(BatchedKernel *table) {
    table[KT_FILL_U32] = batched_kernel<FillU32Params, fill_u32_body, FILL_THREADS, 64>();
    table[KT_FILL_F64] = batched_kernel<FillF64Params, fill_f64_body, FILL_THREADS, 64>();
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
    r->pairs = (double)q->T * q->n_sim * q->n_obs;
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
    for (auto &sl : S->slots) release_slot(sl);
    delete S;
}

}  // namespace dc
