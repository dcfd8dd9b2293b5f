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
// Memory.  Device memory of requests comes from a pool of large segments held against the
// context's HBM budget: a request is admitted when a region of its size can be carved from the
// segments, or a new segment fits under the budget; its region returns to the pool (not to the
// device) when its batch completes.  Segments are only released when no request is in flight, so
// the scheduler thread never frees device memory while batches run.  Host inputs are copied at
// submit into pinned staging (a second pool, host memory) laid out like the front of the
// request's device region, so each request is uploaded with one copy and the scheduler thread
// never copies request data itself; results come back the same way into pinned staging, and
// dc_poll moves them into the caller's buffers.  An event marks the batch's completion.  Every
// request executes exactly the launches of its direct calls, so its results do not depend on
// what it is batched with.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
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
// searches may use any of the three queries-per-lane variants; each sort is either the one-launch
// sort of small segments or up to four 8-bit digit passes (keys below 2^32).
#define SORT_PASSES                                                                          \
    KT_SS_SMALL, KT_SS_HIST, KT_SS_SCAN, KT_SS_SCATTER, KT_SS_HIST, KT_SS_SCAN, KT_SS_SCATTER, \
        KT_SS_HIST, KT_SS_SCAN, KT_SS_SCATTER, KT_SS_HIST, KT_SS_SCAN, KT_SS_SCATTER
const int PROGRAM[] = {
    KT_FILL_U32,  KT_AREA_CDF, KT_SAMPLE,                                      // sampling
    KT_NORM_MAX,  KT_NORM_MAX, KT_PACK,     KT_SCREEN, KT_SCREEN_ROWS, KT_REFINE,  // screen
    KT_BIDIR8,    KT_BIDIR4,   KT_NN_MERGE, KT_BIDIR_MERGE,  // exact, both directions in one pass
    KT_NN8,       KT_NN4,      KT_NN1,      KT_NN_MERGE,   // exact a -> b (or its heavy rows)
    KT_COLMERGE,  KT_COLREFINE,                            // screen, columns
    KT_NN8,       KT_NN4,      KT_NN1,      KT_NN_MERGE,   // exact b -> a (or its heavy columns)
    KT_LOSS,      KT_FILL_F64, SORT_PASSES, KT_BOUNDS, KT_CHAMFER_BWD,         // Chamfer bwd
    SORT_PASSES,  KT_BOUNDS,   SORT_PASSES, KT_BOUNDS,  KT_FACE_GRAD, KT_VERTEX_GRAD};
#undef SORT_PASSES
constexpr int NPROG = (int)(sizeof(PROGRAM) / sizeof(PROGRAM[0]));
static_assert(NPROG <= MAX_STAGES, "program longer than the descriptor");

enum { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2 };

// ---------------------------------------------------------------- segment pools
// Free ranges of one segment: first fit, neighbouring free ranges merged on release.
class RangeList {
  public:
    void init(size_t cap) {
        free_.clear();
        free_[0] = cap;
    }
    bool take(size_t n, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, o = it->first;
            free_.erase(it);
            if (rest) free_[o + n] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t n) {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Segment {
    char *base = nullptr;
    size_t cap = 0;
    RangeList ranges;
};

struct Block {
    char *p = nullptr;
    size_t bytes = 0;
    Segment *seg = nullptr;
};

// A pool of segments (device or pinned host memory); the owner allocates and frees segments.
struct SegPool {
    std::vector<std::unique_ptr<Segment>> segs;
    bool carve(size_t n, Block *b) {
        n = Arena::need(n, 1);
        for (auto &sg : segs) {
            size_t off = 0;
            if (sg->ranges.take(n, &off)) {
                b->p = sg->base + off;
                b->bytes = n;
                b->seg = sg.get();
                return true;
            }
        }
        return false;
    }
    void release(Block *b) {
        if (!b->seg) return;
        b->seg->ranges.give((size_t)(b->p - b->seg->base), b->bytes);
        *b = Block();
    }
    Segment *add(char *base, size_t cap) {
        segs.emplace_back(new Segment());
        Segment *sg = segs.back().get();
        sg->base = base;
        sg->cap = cap;
        sg->ranges.init(cap);
        return sg;
    }
};

constexpr size_t MIB = size_t(1) << 20;
constexpr size_t HOST_SEG_MIN = 64 * MIB;     // first pinned staging segment
constexpr size_t HOST_SEG_MAX = 1024 * MIB;   // segments double up to this size
constexpr size_t DEV_SEG_MIN = 256 * MIB;     // device segments: budget / 8 within these bounds
constexpr size_t DEV_SEG_MAX = 4096 * MIB;

// ---------------------------------------------------------------- request layout
// Byte offsets of a request's pieces within its device region: inputs, then outputs, then the
// intermediates and scratch.  The inputs form one contiguous prefix (one upload) and the outputs
// the next contiguous range (one download).
struct RegionMap {
    size_t verts, faces, obs, fw, loss, status, gverts, pts, bary, fidx, da, ia, db, ib, gl, gpts,
        scratch;
    size_t in_bytes, out_bytes, total;
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

RegionMap region_map(int T, int V, int F, int Na, int Nb, int precision, bool want_grad) {
    const size_t TV = (size_t)T * V, TA = (size_t)T * Na, TB = (size_t)T * Nb;
    RegionMap m;
    size_t off = 0;
    auto take = [&](size_t count, size_t elem) {
        const size_t o = off;
        off += Arena::need(count, elem);
        return o;
    };
    m.verts = take(TV * 3, 4);
    m.faces = take((size_t)F * 3, 4);
    m.obs = take(TB * 3, 4);
    m.fw = take(T, 4);
    m.in_bytes = off;
    m.loss = take(T, 8);
    m.status = take(4, 4);
    m.gverts = want_grad ? take(TV * 3, 4) : off;
    m.out_bytes = off - m.in_bytes;
    m.pts = take(TA * 3, 4);
    m.bary = take(TA * 3, 4);
    m.fidx = take(TA, 4);
    m.da = take(TA, 4);
    m.ia = take(TA, 4);
    m.db = take(TB, 4);
    m.ib = take(TB, 4);
    m.gl = want_grad ? take(T, 8) : off;
    m.gpts = want_grad ? take(TA * 3, 4) : off;
    m.scratch = take(scratch_bytes(T, V, F, Na, Nb, precision, want_grad), 1);
    m.total = off;
    return m;
}

// device pieces of one request at `base`
struct Layout {
    float *verts, *obs, *fw, *pts, *bary, *da, *db, *gpts, *gverts;
    int32_t *faces, *fidx, *ia, *ib;
    double *loss, *gl;
    unsigned *status;
    char *scratch;
};

Layout layout_at(const RegionMap &m, char *base, bool want_grad) {
    Layout L;
    L.verts = reinterpret_cast<float *>(base + m.verts);
    L.faces = reinterpret_cast<int32_t *>(base + m.faces);
    L.obs = reinterpret_cast<float *>(base + m.obs);
    L.fw = reinterpret_cast<float *>(base + m.fw);
    L.loss = reinterpret_cast<double *>(base + m.loss);
    L.status = reinterpret_cast<unsigned *>(base + m.status);
    L.gverts = want_grad ? reinterpret_cast<float *>(base + m.gverts) : nullptr;
    L.pts = reinterpret_cast<float *>(base + m.pts);
    L.bary = reinterpret_cast<float *>(base + m.bary);
    L.fidx = reinterpret_cast<int32_t *>(base + m.fidx);
    L.da = reinterpret_cast<float *>(base + m.da);
    L.ia = reinterpret_cast<int32_t *>(base + m.ia);
    L.db = reinterpret_cast<float *>(base + m.db);
    L.ib = reinterpret_cast<int32_t *>(base + m.ib);
    L.gl = want_grad ? reinterpret_cast<double *>(base + m.gl) : nullptr;
    L.gpts = want_grad ? reinterpret_cast<float *>(base + m.gpts) : nullptr;
    L.scratch = base + m.scratch;
    return L;
}

struct Req {
    uint64_t ticket = 0;
    dc_result *out = nullptr;
    int T = 0, V = 0, F = 0, Na = 0, Nb = 0, precision = 0, reduction = 0;
    uint64_t seed = 0;
    bool want_grad = false, has_w = false;
    RegionMap map{};
    double pairs = 0;
    int state = Q_QUEUED;
    int status = DC_OK;
    Block dev;          // device region, from admission to the batch's completion
    Block h_in, h_out;  // pinned staging, from submit to the final poll
    std::vector<OpRec> ops;
    std::vector<int> stage_of;
};

// the launches of a request's whole pipeline, issued through dispatch()
int issue_request(const Req *r, const Layout &L, unsigned long long *stats) {
    const int T = r->T, V = r->V, F = r->F, Na = r->Na, Nb = r->Nb;
    hipStream_t s = nullptr;  // unused while recording
    fill_u32(L.status, 4, 0u, s);
    Arena sar;
    sar.base = L.scratch;
    sar.cap = r->map.total - r->map.scratch;
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

// record a request's launches against its device region and assign them to program stages
int plan_request(Req *r, unsigned long long *stats) {
    Recording rec;
    g_record = &rec;
    const int rc = issue_request(r, layout_at(r->map, r->dev.p, r->want_grad), stats);
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

// one batch slot: a stream and the captured program over the slot's descriptor
struct BatchSlot {
    hipStream_t stream = nullptr;
    BatchDesc *d_desc = nullptr;
    BatchDesc *h_desc = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t nodes[MAX_STAGES] = {};
    bool enabled[MAX_STAGES] = {};
    int grid[MAX_STAGES] = {};  // workgroups each node launches now
    hipEvent_t ev = nullptr;
    std::vector<Req *> reqs;
    bool busy = false;
};

}  // namespace

// Host copies between the caller's buffers and pinned staging (request inputs at submit, vertex
// gradients at poll): a copy of COPY_SPLIT_MIN bytes or more is cut into pieces of at least
// COPY_PIECE_MIN bytes that a few worker threads copy beside the calling thread, which takes the
// first piece and waits for the rest.  One thread's memcpy would bound the serving loop's
// capacity: a mix of requests carries about a gigabyte of inputs.
constexpr size_t COPY_SPLIT_MIN = size_t(1) << 20;
constexpr size_t COPY_PIECE_MIN = size_t(1) << 19;
constexpr int COPY_WORKERS = 7;

struct CopyPool {
    struct Piece {
        char *dst;
        const char *src;
        size_t n;
        std::atomic<int> *left;
    };
    std::mutex mu;
    std::condition_variable cv, done;
    std::deque<Piece> q;
    std::vector<std::thread> th;
    bool stop = false;

    void start() {
        for (int k = 0; k < COPY_WORKERS; ++k) th.emplace_back([this] { work(); });
    }
    void finish() {
        {
            std::lock_guard<std::mutex> g(mu);
            stop = true;
        }
        cv.notify_all();
        for (auto &t : th) t.join();
        th.clear();
    }
    void work() {
        for (;;) {
            Piece p;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [this] { return stop || !q.empty(); });
                if (q.empty()) return;
                p = q.front();
                q.pop_front();
            }
            std::memcpy(p.dst, p.src, p.n);
            if (p.left->fetch_sub(1) == 1) {
                std::lock_guard<std::mutex> g(mu);
                done.notify_all();
            }
        }
    }
    void copy(void *dst, const void *src, size_t n) {
        char *d = static_cast<char *>(dst);
        const char *s = static_cast<const char *>(src);
        if (n < COPY_SPLIT_MIN || th.empty()) {
            std::memcpy(d, s, n);
            return;
        }
        const size_t k = std::min<size_t>(th.size() + 1, n / COPY_PIECE_MIN);
        const size_t per = (n + k - 1) / k;
        std::atomic<int> left((int)k - 1);
        {
            std::lock_guard<std::mutex> g(mu);
            for (size_t i = 1; i < k; ++i)
                q.push_back({d + i * per, s + i * per, std::min(per, n - i * per), &left});
        }
        cv.notify_all();
        std::memcpy(d, s, per);
        std::unique_lock<std::mutex> lk(mu);
        done.wait(lk, [&left] { return left.load() == 0; });
    }
};

struct Scheduler {
    dc_ctx *ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::condition_variable finished;  // a request reached Q_DONE (dc_wait sleeps on it)
    std::deque<Req *> queue;
    std::unordered_map<uint64_t, Req *> table;
    uint64_t next_ticket = 1;
    int running = 0;  // requests admitted and not finished on the device
    bool stop = false;
    BatchedKernel kern[KT_COUNT] = {};
    BatchSlot slots[NSLOTS];
    std::thread th;
    CopyPool copies;  // host copies of request inputs and results
    // device memory of admitted requests (scheduler thread only)
    SegPool dpool;
    size_t dev_seg = DEV_SEG_MIN;
    // pinned staging of requests between submit and poll
    std::mutex hmu;
    SegPool hpool;
    size_t host_seg = HOST_SEG_MIN;
};

size_t request_bytes(int T, int V, int F, int Na, int Nb, int precision, bool want_grad) {
    return region_map(T, V, F, Na, Nb, precision, want_grad).total;
}

size_t serving_fixed_bytes() { return sizeof(BatchDesc) * NSLOTS; }

// pinned staging for `n` bytes; a new segment is added when none has room (client threads only)
static int host_alloc(Scheduler *S, size_t n, Block *b) {
    std::lock_guard<std::mutex> g(S->hmu);
    if (S->hpool.carve(n, b)) return DC_OK;
    const size_t want = std::max(Arena::need(n, 1), S->host_seg);
    void *p = nullptr;
    if (hipHostMalloc(&p, want, 0) != hipSuccess) {
        (void)hipGetLastError();
        set_error("pinned staging allocation failed");
        return DC_ERR_NOMEM;
    }
    S->hpool.add(static_cast<char *>(p), want);
    S->host_seg = std::min(S->host_seg * 2, HOST_SEG_MAX);
    return S->hpool.carve(n, b) ? DC_OK : DC_ERR_NOMEM;
}

static void host_release(Scheduler *S, Block *b) {
    std::lock_guard<std::mutex> g(S->hmu);
    S->hpool.release(b);
}

// Add a device segment that holds `need` bytes, counted against the budget: the default segment
// size when it fits, else whatever the budget still allows.  DC_ERR_BUDGET when the budget has
// no room for `need`; DC_ERR_NOMEM when the device refuses the allocation.
static int dev_grow(Scheduler *S, size_t need, bool exact) {
    dc_ctx *ctx = S->ctx;
    size_t room;
    {
        std::lock_guard<std::mutex> g(ctx->budget_mu);
        room = ctx->budget - ctx->held;
    }
    need = Arena::need(need, 1);
    if (need > room) {
        set_error("request of " + std::to_string(need) + " bytes does not fit the budget (" +
                  std::to_string(room) + " bytes free)");
        return DC_ERR_BUDGET;
    }
    const size_t want = exact ? need : std::min(std::max(need, S->dev_seg), room);
    void *p = nullptr;
    const int rc = dev_alloc_raw(ctx, &p, want);
    if (rc != DC_OK) return rc;
    S->dpool.add(static_cast<char *>(p), want);
    return DC_OK;
}

// give the device segments back (only while no request is in flight: every segment is free)
static void dev_release_all(Scheduler *S) {
    for (auto &sg : S->dpool.segs) dev_free(S->ctx, sg->base, sg->cap);
    S->dpool.segs.clear();
}

// A queued request's device region and plan.  DC_OK: admitted; DC_PENDING: not now (memory
// returns when requests in flight finish); an error: the request fails alone.
static int admit(Scheduler *S, Req *r) {
    if (forced_alloc_failure(S->ctx)) {
        set_error("device region of a request: allocation failed (forced)");
        return DC_ERR_NOMEM;
    }
    const size_t n = r->map.total;
    if (!S->dpool.carve(n, &r->dev)) {
        int rc = dev_grow(S, n, false);
        if (rc != DC_OK) {
            if (S->running > 0) return DC_PENDING;
            // nothing in flight, so every segment is free and none is large enough: trade them
            // for one that holds this request exactly
            dev_release_all(S);
            rc = dev_grow(S, n, true);
            if (rc != DC_OK) return rc;
        }
        if (!S->dpool.carve(n, &r->dev)) {
            set_error("device pool: a new segment could not hold its request");
            return DC_ERR_NOMEM;
        }
    }
    const int rc = plan_request(r, S->ctx->d_stats);
    if (rc != DC_OK) S->dpool.release(&r->dev);
    return rc;
}

// a request leaves the device: its status word is read from its staging, its region returns to
// the pool; dc_poll hands the results over
static void finish_req(Scheduler *S, Req *r, bool on_device) {
    if (on_device) {
        if (r->status == DC_OK) {
            unsigned st = 0;
            std::memcpy(&st, r->h_out.p + (r->map.status - r->map.in_bytes), 4);
            if (st & ST_BAD_FACE)
                r->status = DC_ERR_INVALID;
            else if (st & ST_DEGENERATE)
                r->status = DC_ERR_DEGENERATE;
        }
        S->dpool.release(&r->dev);
        --S->running;
    }
    r->state = Q_DONE;
    std::vector<OpRec>().swap(r->ops);
    S->finished.notify_all();
}

// workgroups of a stage's node: its persistent grid, or fewer when the batch has less work
static int stage_grid(const BatchedKernel &k, int total) {
    int g = 1;
    while (g < total && g < k.blocks) g <<= 1;
    return std::min(g, k.blocks);
}

// stage `st` of the slot's graph as a kernel node of `blocks` workgroups: added to the graph
// (building it) or set in the executable graph (the slot idle)
static int set_stage_params(Scheduler *S, BatchSlot &sl, int st, int blocks, bool exec) {
    const BatchedKernel &k = S->kern[PROGRAM[st]];
    const BatchDesc *desc = sl.d_desc;
    int stage = st;
    void *args[2] = {&desc, &stage};
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void *>(k.func);
    kp.gridDim = dim3(blocks);
    kp.blockDim = dim3(k.threads);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    if (exec)
        DC_HIP(hipGraphExecKernelNodeSetParams(sl.exec, sl.nodes[st], &kp));
    else
        DC_HIP(hipGraphAddKernelNode(&sl.nodes[st], sl.graph, st ? &sl.nodes[st - 1] : nullptr,
                                     st ? 1 : 0, &kp));
    sl.grid[st] = blocks;
    return DC_OK;
}

// upload, replay and download one batch on slot `sl`; on failure every request of the batch
// fails with the returned status
static int run_batch(Scheduler *S, BatchSlot &sl) {
    hipStream_t s = sl.stream;
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
    // inputs: one copy per request from its pinned staging (laid out like its region's front)
    for (Req *r : sl.reqs)
        DC_HIP(hipMemcpyAsync(r->dev.p + r->map.verts, r->h_in.p, r->map.in_bytes,
                              hipMemcpyHostToDevice, s));
    const size_t dsz = sizeof(D->stage) + (size_t)nops * sizeof(OpRec);
    DC_HIP(hipMemcpyAsync(sl.d_desc, D, dsz, hipMemcpyHostToDevice, s));
    // stages without work in this batch are switched off, and the others launch no more
    // workgroups than the power of two at or above their logical workgroups (every persistent
    // workgroup costs launch time even when it finds nothing to do); the slot is idle, so its
    // executable graph may be updated
    for (int st = 0; st < NPROG; ++st) {
        const int total = D->stage[st].total;
        const bool on = total > 0;
        if (on != sl.enabled[st]) {
            DC_HIP(hipGraphNodeSetEnabled(sl.exec, sl.nodes[st], on ? 1u : 0u));
            sl.enabled[st] = on;
        }
        if (!on) continue;
        const int want = stage_grid(S->kern[PROGRAM[st]], total);
        if (want != sl.grid[st]) {
            const int rc = set_stage_params(S, sl, st, want, true);
            if (rc != DC_OK) return rc;
        }
    }
    DC_HIP(hipGraphLaunch(sl.exec, s));
    for (Req *r : sl.reqs)
        DC_HIP(hipMemcpyAsync(r->h_out.p, r->dev.p + r->map.in_bytes, r->map.out_bytes,
                              hipMemcpyDeviceToHost, s));
    DC_HIP(hipEventRecord(sl.ev, s));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "serving batch launch");
    return DC_OK;
}

static void fail_batch(Scheduler *S, BatchSlot &sl, int rc) {
    (void)hipStreamSynchronize(sl.stream);  // anything already enqueued has finished
    for (Req *r : sl.reqs) {
        r->status = rc;
        finish_req(S, r, true);
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
        const int rc = admit(S, r);
        if (rc == DC_PENDING) break;
        S->queue.pop_front();
        r->out->t_admit = now_s();
        if (rc != DC_OK) {  // this request alone fails
            r->status = rc;
            finish_req(S, r, false);
            continue;
        }
        ++S->running;
        r->state = Q_RUNNING;
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
        // completions first: their memory may admit the next requests
        for (auto &sl : S->slots) {
            if (!sl.busy || hipEventQuery(sl.ev) != hipSuccess) continue;
            for (Req *r : sl.reqs) finish_req(S, r, true);
            sl.reqs.clear();
            sl.busy = false;
            progressed = true;
        }
        for (auto &sl : S->slots) {
            if (sl.busy) continue;
            if (!form_batch(S, sl)) {
                if (S->queue.empty()) break;
                continue;
            }
            sl.busy = true;
            progressed = true;
            // launching runs unlocked: the slot and its requests belong to this thread until
            // they finish, and submit / poll only touch the queue and the table
            lk.unlock();
            const int rc = run_batch(S, sl);
            lk.lock();
            if (rc != DC_OK) fail_batch(S, sl, rc);
        }
        if (progressed) continue;
        bool busy = false;
        for (auto &sl : S->slots) busy |= sl.busy;
        if (busy) {
            // a batch is on the device: look at its event again at once (a timed wait would add
            // its wake-up delay to every request's latency)
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            S->cv.wait_for(lk, std::chrono::microseconds(50));
        }
    }
}

static int init_slot(Scheduler *S, BatchSlot &sl) {
    DC_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    DC_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    void *p = nullptr;
    const int rc = dev_alloc_raw(S->ctx, &p, sizeof(BatchDesc));
    if (rc != DC_OK) return rc;
    sl.d_desc = static_cast<BatchDesc *>(p);
    DC_HIP(hipHostMalloc(reinterpret_cast<void **>(&sl.h_desc), sizeof(BatchDesc), 0));
    // an empty descriptor: a replay before the first upload does nothing
    std::memset(sl.h_desc, 0, sizeof(BatchDesc));
    DC_HIP(hipMemcpy(sl.d_desc, sl.h_desc, sizeof(sl.h_desc->stage), hipMemcpyHostToDevice));
    // the program as a chain of kernel nodes over the slot's descriptor
    DC_HIP(hipGraphCreate(&sl.graph, 0));
    for (int st = 0; st < NPROG; ++st) {
        const int rc = set_stage_params(S, sl, st, S->kern[PROGRAM[st]].blocks, false);
        if (rc != DC_OK) return rc;
        sl.enabled[st] = true;
    }
    DC_HIP(hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0));
    return DC_OK;
}

static void release_slot(dc_ctx *ctx, BatchSlot &sl) {
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    if (sl.graph) (void)hipGraphDestroy(sl.graph);
    if (sl.d_desc) dev_free(ctx, sl.d_desc, sizeof(BatchDesc));
    if (sl.h_desc) (void)hipHostFree(sl.h_desc);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    sl = BatchSlot();
}

static void release_pools(Scheduler *S) {
    dev_release_all(S);
    for (auto &sg : S->hpool.segs) (void)hipHostFree(sg->base);
    S->hpool.segs.clear();
}

static int ensure_scheduler(dc_ctx *ctx) {
    if (ctx->sched) return DC_OK;
    Scheduler *S = new Scheduler();
    S->ctx = ctx;
    S->dev_seg = std::min(std::max(ctx->budget / 8, DEV_SEG_MIN), DEV_SEG_MAX);
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
        for (auto &sl : S->slots) release_slot(ctx, sl);
        delete S;
        return rc;
    }
    S->copies.start();
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
    const RegionMap map =
        region_map(q->T, q->V, q->F, q->n_sim, q->n_obs, q->precision, want_grad);
    if (map.total + serving_fixed_bytes() + CTX_WORDS_BYTES > ctx->budget) {
        set_error("dc_submit: request needs " + std::to_string(map.total) +
                  " bytes, more than the budget holds beside the serving loop's descriptors");
        return DC_ERR_BUDGET;
    }
    Scheduler *S = nullptr;
    {
        std::lock_guard<std::mutex> g(ctx->mu);  // creation of the loop is serialised with direct calls
        const int rc = ensure_scheduler(ctx);
        if (rc) return rc;
        S = ctx->sched;
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
    r->has_w = q->frame_w != nullptr;
    r->map = map;
    r->pairs = (double)q->T * q->n_sim * q->n_obs;
    // the inputs go straight into pinned staging laid out like the region's input prefix
    int rc = host_alloc(S, map.in_bytes, &r->h_in);
    if (rc == DC_OK) rc = host_alloc(S, map.out_bytes, &r->h_out);
    if (rc != DC_OK) {
        host_release(S, &r->h_in);
        delete r;
        return rc;
    }
    char *h = r->h_in.p;
    S->copies.copy(h + map.verts, q->verts, (size_t)q->T * q->V * 3 * 4);
    S->copies.copy(h + map.faces, q->faces, (size_t)q->F * 3 * 4);
    S->copies.copy(h + map.obs, q->observed, (size_t)q->T * q->n_obs * 3 * 4);
    if (r->has_w) std::memcpy(h + map.fw, q->frame_w, (size_t)q->T * 4);
    out->t_submit = now_s();
    out->t_admit = 0;
    out->t_done = 0;
    out->status = DC_PENDING;
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

// the results of a finished request (removed from the table) into the caller's buffers
static int hand_over(Scheduler *S, Req *r, const char *who) {
    const char *h = r->h_out.p;
    if (r->status == DC_OK) {
        std::memcpy(r->out->loss, h + (r->map.loss - r->map.in_bytes), (size_t)r->T * 8);
        if (r->want_grad)
            S->copies.copy(r->out->grad_verts, h + (r->map.gverts - r->map.in_bytes),
                           (size_t)r->T * r->V * 3 * 4);
    }
    const int st = r->status;
    r->out->status = st;
    r->out->t_done = now_s();
    host_release(S, &r->h_in);
    host_release(S, &r->h_out);
    delete r;
    if (st != DC_OK) set_error(std::string(who) + ": the request failed");
    return st;
}

// wait up to timeout_us (< 0: without limit, 0: not at all) for the ticket's request, then hand
// its results over
static int wait_for_ticket(dc_ctx *ctx, uint64_t ticket, long long timeout_us, const char *who) {
    Scheduler *S = ctx->sched;
    if (!S) {
        set_error(std::string(who) + ": unknown ticket");
        return DC_ERR_INVALID;
    }
    Req *r = nullptr;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        const auto deadline =
            std::chrono::steady_clock::now() + std::chrono::microseconds(std::max(timeout_us, 0LL));
        for (;;) {
            auto it = S->table.find(ticket);
            if (it == S->table.end()) {
                set_error(std::string(who) + ": unknown ticket");
                return DC_ERR_INVALID;
            }
            if (it->second->state == Q_DONE) {
                r = it->second;
                S->table.erase(it);
                break;
            }
            if (timeout_us == 0) return DC_PENDING;
            if (timeout_us < 0)
                S->finished.wait(lk);
            else if (S->finished.wait_until(lk, deadline) == std::cv_status::timeout &&
                     S->table.count(ticket) && S->table[ticket]->state != Q_DONE)
                return DC_PENDING;
        }
    }
    // the request now belongs to this thread: hand its results over outside the scheduler's lock
    return hand_over(S, r, who);
}

int sched_poll(dc_ctx *ctx, uint64_t ticket) { return wait_for_ticket(ctx, ticket, 0, "dc_poll"); }

int sched_wait(dc_ctx *ctx, uint64_t ticket, long long timeout_us) {
    return wait_for_ticket(ctx, ticket, timeout_us, "dc_wait");
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
    S->copies.finish();
    for (auto &kv : S->table) delete kv.second;
    for (auto &sl : S->slots) release_slot(ctx, sl);
    release_pools(S);
    delete S;
}

}  // namespace dc
