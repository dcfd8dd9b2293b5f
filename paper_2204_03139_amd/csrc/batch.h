// Launch plumbing shared by direct calls and the batched serving pipeline.
//
// Every kernel of the hot path is written as a body over one logical workgroup (Blk) of a logical
// grid, with its arguments in a plain parameter struct.  A direct call launches the body on the
// hardware grid.  The serving loop instead records, per request, the sequence of (kernel, grid,
// parameters) that the same host code would launch, lays the records of a whole batch of
// requests out in a device descriptor, and replays one captured graph of persistent kernels over
// it: stage s of the graph runs, for every request of the batch, that request's s-th recorded
// launch, each workgroup walking the stage's flattened list of logical workgroups.  A request
// therefore executes exactly the arithmetic of its direct launches, whatever else is batched
// with it.
#pragma once

#include <cstring>
#include <type_traits>
#include <vector>

#include "dc_internal.h"

namespace dc {

// one logical workgroup of a logical grid
struct Blk {
    int x, y, z, gx, gy, gz;
};

__device__ __forceinline__ Blk grid_blk() {
    Blk b;
    b.x = blockIdx.x;
    b.y = blockIdx.y;
    b.z = blockIdx.z;
    b.gx = gridDim.x;
    b.gy = gridDim.y;
    b.gz = gridDim.z;
    return b;
}

// The same logical (x, y) grid with the workgroups of each XCD kept together: the hardware deals
// workgroups out to the 8 XCDs in turn (flat id modulo 8), so XCD k is given the k-th contiguous
// eighth of the frame-major order.  Each XCD's L2 then holds the data of the one or two frames its
// workgroups are on, instead of every XCD touching every frame in flight.  A bijection on the
// workgroups of the grid (x fastest, then y, then z); only the mapping, never the work, changes.
constexpr unsigned NUM_XCD = 8;
__device__ __forceinline__ Blk grid_blk_xcd() {
    const unsigned gx = gridDim.x, gxy = gridDim.x * gridDim.y, total = gxy * gridDim.z;
    const unsigned b = blockIdx.x + gx * blockIdx.y + gxy * blockIdx.z;
    const unsigned per = total / NUM_XCD, rem = total % NUM_XCD;
    const unsigned xcd = b % NUM_XCD, k = b / NUM_XCD;
    const unsigned l = xcd * per + (xcd < rem ? xcd : rem) + k;
    Blk r;
    r.x = (int)(l % gx);
    r.y = (int)((l % gxy) / gx);
    r.z = (int)(l / gxy);
    r.gx = (int)gx;
    r.gy = (int)gridDim.y;
    r.gz = (int)gridDim.z;
    return r;
}

// kernels that can be recorded (one batched persistent kernel each)
enum KernelType : int {
    KT_FILL_U32 = 0,
    KT_FILL_F64,
    KT_AREA_CDF,
    KT_SAMPLE,
    KT_NORM_MAX,
    KT_PACK,
    KT_SCREEN,
    KT_SCREEN_ROWS,
    KT_REFINE,
    KT_COLMERGE,
    KT_COLREFINE,
    KT_NN1,
    KT_NN4,
    KT_NN8,
    KT_NN_MERGE,
    KT_LOSS,
    KT_SS_HIST,
    KT_SS_SCAN,
    KT_SS_SCATTER,
    KT_CHAMFER_BWD,
    KT_BOUNDS,
    KT_FACE_GRAD,
    KT_VERTEX_GRAD,
    KT_BIDIR8,
    KT_BIDIR4,
    KT_BIDIR_MERGE,
    KT_SS_SMALL,
    KT_COUNT
};

constexpr int OP_PARAM_BYTES = 144;

// one recorded launch; in the device descriptor `start` is the op's first flattened workgroup
// within its stage
struct OpRec {
    int start, gx, gy, gz;
    alignas(16) unsigned char p[OP_PARAM_BYTES];
};

constexpr int MAX_STAGES = 72;   // length of the serving program
constexpr int MAX_BATCH = 32;    // requests per batch
constexpr int MAX_OPS = MAX_STAGES * MAX_BATCH;

struct StageHdr {
    int total;  // flattened workgroups of the stage over the batch
    int first;  // first op of the stage
    int nops;
    int pad;
};

struct BatchDesc {
    StageHdr stage[MAX_STAGES];
    OpRec op[MAX_OPS];
};

// host: while non-null, launches made through dispatch() on this thread are recorded here
// (with their kernel type in the parallel vector) instead of being executed
struct Recording {
    std::vector<OpRec> ops;
    std::vector<int> types;
};
extern thread_local Recording *g_record;

template <class P>
inline void dispatch(int type, void (*kern)(P), dim3 grid, int threads, const P &p,
                     hipStream_t s) {
    static_assert(sizeof(P) <= OP_PARAM_BYTES, "parameter block too large to record");
    static_assert(std::is_trivially_copyable<P>::value, "parameters must be plain data");
    if (g_record) {
        if ((long)grid.x * grid.y * grid.z == 0) return;
        OpRec o;
        std::memset(&o, 0, sizeof(o));
        o.gx = (int)grid.x;
        o.gy = (int)grid.y;
        o.gz = (int)grid.z;
        std::memcpy(o.p, &p, sizeof(P));
        g_record->ops.push_back(o);
        g_record->types.push_back(type);
        return;
    }
    hipLaunchKernelGGL(kern, grid, dim3(threads), 0, s, p);
}

// a block-uniform value read from memory, kept in scalar registers
__device__ __forceinline__ int uniform_int(const int *p) { return __builtin_amdgcn_readfirstlane(*p); }

template <class P>
__device__ __forceinline__ P uniform_params(const unsigned char *src) {
    static_assert(sizeof(P) % 4 == 0, "parameter blocks are whole words");
    P out;
    int *o = reinterpret_cast<int *>(&out);
    const int *w = reinterpret_cast<const int *>(src);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(P) / 4); ++k) o[k] = __builtin_amdgcn_readfirstlane(w[k]);
    return out;
}

// device: walk the flattened logical workgroups of one stage
template <class P, void (*BODY)(const P &, const Blk &)>
__device__ __forceinline__ void run_stage(const BatchDesc *__restrict__ d, int stage) {
    const int total = uniform_int(&d->stage[stage].total);
    const int first = uniform_int(&d->stage[stage].first);
    const int nops = uniform_int(&d->stage[stage].nops);
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        int lo = first, hi = first + nops - 1;
        while (lo < hi) {  // last op whose start is <= item
            const int mid = (lo + hi + 1) >> 1;
            if (uniform_int(&d->op[mid].start) <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const OpRec &o = d->op[lo];
        const int local = item - uniform_int(&o.start);
        Blk b;
        b.gx = uniform_int(&o.gx);
        b.gy = uniform_int(&o.gy);
        b.gz = uniform_int(&o.gz);
        b.x = local % b.gx;
        const int rest = local / b.gx;
        b.y = rest % b.gy;
        b.z = rest / b.gy;
        const P p = uniform_params<P>(o.p);
        BODY(p, b);
        __syncthreads();  // the next item may reuse the body's LDS
    }
}

// the batched persistent kernel of one body (MINW: waves per SIMD the registers must allow)
template <class P, void (*BODY)(const P &, const Blk &), int THREADS, int MINW>
__global__ __launch_bounds__(THREADS, MINW) void k_batched(const BatchDesc *__restrict__ d,
                                                           int stage) {
    run_stage<P, BODY>(d, stage);
}

// a batched kernel as a graph node: its function and launch shape
struct BatchedKernel {
    const void *func = nullptr;
    int threads = 0;
    int blocks = 0;
};

template <class P, void (*BODY)(const P &, const Blk &), int THREADS, int BLOCKS, int MINW = 1>
BatchedKernel batched_kernel() {
    BatchedKernel k;
    k.func = reinterpret_cast<const void *>(&k_batched<P, BODY, THREADS, MINW>);
    k.threads = THREADS;
    k.blocks = BLOCKS;
    return k;
}

// each kernel file fills the entries of its kernel types
void register_sample_kernels(BatchedKernel *table);
void register_nn_kernels(BatchedKernel *table);
void register_screen_kernels(BatchedKernel *table);
void register_sort_kernels(BatchedKernel *table);
void register_backward_kernels(BatchedKernel *table);
void register_fill_kernels(BatchedKernel *table);

}  // namespace dc
