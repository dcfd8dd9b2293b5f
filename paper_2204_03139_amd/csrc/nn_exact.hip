// Exact single-precision nearest neighbours (the plain fp32 path of Sec. III-A, Eq. 1/2) and the
// per-frame loss reduction.
//
// k_nn_exact: each lane owns QPT queries held in registers; the workgroup streams the target
// cloud through LDS in tiles of NN_TILE points (one 16-byte broadcast read per target per lane).
// Per pair the lane evaluates the canonical distance fma(dz,dz,fma(dy,dy,dx*dx)) and keeps only a
// running minimum over a sub-tile of NN_SUB targets (one v_min per pair); the first sub-tile with
// a strictly smaller minimum is remembered.  At the end the lane rescans that one sub-tile from
// global memory for the first index whose distance equals the minimum, which is the smallest
// index among the exact ties, so the result is the exact argmin with the smallest-index rule.
// Large frames split the target range over grid.z slices; a merge kernel combines the slices in
// slice order with the same strict-less rule.
//
// k_nn_bidir: both directions in one pass, each pair's canonical distance evaluated once.  A lane
// owns 8 (or 4) consecutive rows of a; targets b stream through LDS.  Rows keep k_nn_exact's
// sub-tile minima (and its rescan); for the columns each lane folds its rows into one value per
// target, each wave reads its lanes' values of a 16-target block back transposed from its own
// LDS region and reduces them to (minimum, first lane reaching it) as one 64-bit key (distance
// bits, lane), and an LDS atomic minimum combines the four waves.  k_bidir_merge takes the smallest
// key over the row blocks of a frame (the smallest distance, then the first lane in row order) and
// evaluates that lane's rows again for the first one whose distance equals the minimum: the exact
// argmin with the smallest-index rule.  The targets may be split over slices, whose row results
// merge in slice order like k_nn_exact's.
#include <cmath>

#include "batch.h"

namespace dc {
namespace {

constexpr int NN_THREADS = 256;
constexpr int NN_TILE = 1024;
constexpr int NN_SUB = 64;

__device__ __forceinline__ float canon_d2(float qx, float qy, float qz, float px, float py,
                                          float pz) {
    const float dx = qx - px;
    const float dy = qy - py;
    const float dz = qz - pz;
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// qlist/qcount (optional): per frame, only the queries qlist[t*Nq + k], k < qcount[t], are
// searched; slice partials are then indexed by k and the merge maps them back to the rows.
struct NNParams {
    const float *Q;
    const float *P;
    int32_t *idx;
    float *dist;
    const int32_t *qlist;
    const int32_t *qcount;
    size_t slice_stride;
    int Nq, Np, slice_len;
};

// A short query list (the screen's heavy queries): one wave per query, its 64 lanes striding
// over the slice, so a handful of queries still keeps every lane busy.  The result is the one the
// lane-per-query search gives: the smallest index among the minimal distances (fminf order: NaN
// distances never win), and when no distance is below infinity, the first index of the first
// 64-target sub-tile whose distance is infinite, or the slice's first index.
constexpr int NN_SHORT_LIST = 128;

__device__ __noinline__ void short_list_search(const NNParams &pr, int t, int z, int nq_live,
                                               int j_begin, int j_end) {
    const int Nq = pr.Nq, Np = pr.Np;
    const float *Qt = pr.Q + (size_t)t * Nq * 3;
    const float *Pt = pr.P + (size_t)t * Np * 3;
    const int lane = threadIdx.x & 63;
    const float inf = __builtin_inff();
    for (int k = threadIdx.x >> 6; k < nq_live; k += NN_THREADS / 64) {
        const int qi = pr.qlist[(size_t)t * Nq + k];
        const float qx = Qt[3 * (size_t)qi], qy = Qt[3 * (size_t)qi + 1],
                    qz = Qt[3 * (size_t)qi + 2];
        float best = inf;
        int bj = 0x7fffffff;
        // eight targets per lane per step, each read whole (one 12-byte load), the eight loads in
        // flight together; a lane still visits its targets in increasing order
        int j = j_begin + lane;
        for (; j + 7 * 64 < j_end; j += 8 * 64) {
            float c[8][3];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float *p = Pt + 3 * (size_t)(j + 64 * u);
                c[u][0] = p[0];
                c[u][1] = p[1];
                c[u][2] = p[2];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float d = canon_d2(qx, qy, qz, c[u][0], c[u][1], c[u][2]);
                if (d < best) {  // a lane's indices increase: strict-less keeps its first minimum
                    best = d;
                    bj = j + 64 * u;
                }
            }
        }
        for (; j < j_end; j += 64) {
            const float *p = Pt + 3 * (size_t)j;
            const float d = canon_d2(qx, qy, qz, p[0], p[1], p[2]);
            if (d < best) {
                best = d;
                bj = j;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off, 64);
            const int oj = __shfl_xor(bj, off, 64);
            if (ob < best || (ob == best && oj < bj)) {
                best = ob;
                bj = oj;
            }
        }
        if (!(best < inf)) {  // nothing finite: the first infinite distance of the first sub-tile
            const int j = j_begin + lane;
            bool hit = false;
            if (j < min(j_begin + NN_SUB, j_end)) {
                const float *p = Pt + 3 * (size_t)j;
                hit = canon_d2(qx, qy, qz, p[0], p[1], p[2]) == inf;
            }
            const unsigned long long m = __ballot(hit);
            bj = m ? j_begin + (int)__builtin_ctzll(m) : j_begin;
            best = inf;
        }
        if (lane == 0) {
            const size_t o = pr.slice_stride ? (size_t)z * pr.slice_stride + (size_t)t * Nq + k
                                             : (size_t)t * Nq + qi;
            pr.idx[o] = bj;
            pr.dist[o] = best;
        }
    }
}

template <int QPT>
__device__ __forceinline__ void nn_exact_body(const NNParams &pr, const Blk &blk) {
    const float *__restrict__ Q = pr.Q;
    const float *__restrict__ P = pr.P;
    const int Nq = pr.Nq, Np = pr.Np, slice_len = pr.slice_len;
    int32_t *__restrict__ idx = pr.idx;
    float *__restrict__ dist = pr.dist;
    const size_t slice_stride = pr.slice_stride;
    const int32_t *__restrict__ qlist = pr.qlist;
    const int32_t *__restrict__ qcount = pr.qcount;
    __shared__ float4 tile[NN_TILE];
    const int t = blk.y;
    const int z = blk.z;
    const int nq_live = qlist ? qcount[t] : Nq;
    const float *Qt = Q + (size_t)t * Nq * 3;
    const float *Pt = P + (size_t)t * Np * 3;
    const int j_begin = z * slice_len;
    const int j_end = min(Np, j_begin + slice_len);
    if (QPT == 1 && qlist && nq_live <= NN_SHORT_LIST) {
        if (blk.x == 0) short_list_search(pr, t, z, nq_live, j_begin, j_end);
        return;
    }
    // the list of a frame is short and its length only known on the device: each workgroup
    // walks query blocks x, x + gx, ... of its logical grid (one step without a list)
    for (int qb = blk.x; qb * NN_THREADS * QPT < nq_live; qb += blk.gx) {
    const int q0 = qb * NN_THREADS * QPT + threadIdx.x;
    // a wave whose queries all lie past the list end only helps stage the tiles
    const bool wave_live = qb * NN_THREADS * QPT + (int)(threadIdx.x & ~63u) < nq_live;

    float qx[QPT], qy[QPT], qz[QPT], best[QPT];
    int bsub[QPT];
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
        const int qk = q0 + k * NN_THREADS;
        const bool ok = qk < nq_live;
        const int qi = ok ? (qlist ? qlist[(size_t)t * Nq + qk] : qk) : 0;
        qx[k] = ok ? Qt[3 * (size_t)qi] : 0.f;
        qy[k] = ok ? Qt[3 * (size_t)qi + 1] : 0.f;
        qz[k] = ok ? Qt[3 * (size_t)qi + 2] : 0.f;
        best[k] = __builtin_inff();
        bsub[k] = j_begin;
    }

    for (int base = j_begin; base < j_end; base += NN_TILE) {
        const int n = min(NN_TILE, j_end - base);
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += NN_THREADS) {
            const float *p = Pt + 3 * (size_t)(base + j);
            tile[j] = make_float4(p[0], p[1], p[2], 0.f);
        }
        __syncthreads();
        if (!wave_live) continue;
        int s0 = 0;
        for (; s0 + NN_SUB <= n; s0 += NN_SUB) {
            float m[QPT];
#pragma unroll
            for (int k = 0; k < QPT; ++k) m[k] = __builtin_inff();
#pragma unroll 8
            for (int j = s0; j < s0 + NN_SUB; ++j) {
                const float4 p = tile[j];
#pragma unroll
                for (int k = 0; k < QPT; ++k)
                    m[k] = __builtin_fminf(m[k], canon_d2(qx[k], qy[k], qz[k], p.x, p.y, p.z));
            }
#pragma unroll
            for (int k = 0; k < QPT; ++k)
                if (m[k] < best[k]) {
                    best[k] = m[k];
                    bsub[k] = base + s0;
                }
        }
        if (s0 < n) {  // ragged tail of the slice
            float m[QPT];
#pragma unroll
            for (int k = 0; k < QPT; ++k) m[k] = __builtin_inff();
            for (int j = s0; j < n; ++j) {
                const float4 p = tile[j];
#pragma unroll
                for (int k = 0; k < QPT; ++k)
                    m[k] = __builtin_fminf(m[k], canon_d2(qx[k], qy[k], qz[k], p.x, p.y, p.z));
            }
#pragma unroll
            for (int k = 0; k < QPT; ++k)
                if (m[k] < best[k]) {
                    best[k] = m[k];
                    bsub[k] = base + s0;
                }
        }
    }

    // rescan the winning sub-tile for the first exact match
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
        const int qk = q0 + k * NN_THREADS;
        if (qk >= nq_live) continue;
        const int qi = (qlist && slice_stride == 0) ? qlist[(size_t)t * Nq + qk] : qk;
        const int js = bsub[k];
        const int je = min(js + NN_SUB, j_end);
        int found = js;
        for (int j = js; j < je; ++j) {
            const float *p = Pt + 3 * (size_t)j;
            if (canon_d2(qx[k], qy[k], qz[k], p[0], p[1], p[2]) == best[k]) {
                found = j;
                break;
            }
        }
        const size_t o = (size_t)z * slice_stride + (size_t)t * Nq + qi;
        idx[o] = found;
        dist[o] = best[k];
    }
    __syncthreads();  // the next query block restages the tiles
    }
}

template <int QPT>
__global__ __launch_bounds__(NN_THREADS) void k_nn_exact(NNParams p) {
    nn_exact_body<QPT>(p, grid_blk_xcd());
}

// combine per-slice winners; slices hold increasing index ranges, so strict-less keeps the
// smallest index among equal distances.  With a query list, position k of frame t goes back to
// row qlist[t*Nq + k].
struct NNMergeParams {
    const int32_t *pidx;
    const float *pdist;
    int32_t *idx;
    float *dist;
    const int32_t *qlist;
    const int32_t *qcount;
    size_t slice_stride;
    int slices, Nq, T;
};

constexpr int MERGE_THREADS = 256;

__device__ __forceinline__ void nn_merge_body(const NNMergeParams &pr, const Blk &blk) {
    const int32_t *__restrict__ pidx = pr.pidx;
    const float *__restrict__ pdist = pr.pdist;
    const int slices = pr.slices, Nq = pr.Nq, T = pr.T;
    const size_t slice_stride = pr.slice_stride;
    const int32_t *__restrict__ qlist = pr.qlist;
    const int32_t *__restrict__ qcount = pr.qcount;
    const size_t o = (size_t)blk.x * MERGE_THREADS + threadIdx.x;
    if (o >= (size_t)T * Nq) return;
    const int t = (int)(o / Nq);
    const int k = (int)(o - (size_t)t * Nq);
    if (qlist && k >= qcount[t]) return;
    float b = pdist[o];
    int bi = pidx[o];
    for (int z = 1; z < slices; ++z) {
        const float d = pdist[z * slice_stride + o];
        if (d < b) {
            b = d;
            bi = pidx[z * slice_stride + o];
        }
    }
    const size_t out = qlist ? (size_t)t * Nq + qlist[o] : o;
    pr.idx[out] = bi;
    pr.dist[out] = b;
}

__global__ __launch_bounds__(MERGE_THREADS) void k_nn_merge(NNMergeParams p) {
    nn_merge_body(p, grid_blk());
}

constexpr int LOSS_THREADS = 1024;

struct LossParams {
    const float *da;
    const float *db;
    const float *frame_w;
    double *loss;
    double alpha, beta;
    int Na, Nb;
};

// loss[t] = w_t (alpha sum_i dist_a + beta sum_j dist_b), in double, in a fixed order
__device__ __forceinline__ void loss_body(const LossParams &p, const Blk &blk) {
    const float *__restrict__ da = p.da;
    const float *__restrict__ db = p.db;
    const int Na = p.Na, Nb = p.Nb;
    const double alpha = p.alpha, beta = p.beta;
    __shared__ double sa[LOSS_THREADS], sb[LOSS_THREADS];
    const int t = blk.x;
    double xa = 0.0, xb = 0.0;
    // four independent partial sums per thread keep several loads in flight; they are added in
    // a fixed order, as is the tree below, so the result is the same on every run
    auto sum4 = [](const float *x, int n) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int i = threadIdx.x;
        for (; i + 3 * LOSS_THREADS < n; i += 4 * LOSS_THREADS) {
            s0 += (double)x[i];
            s1 += (double)x[i + LOSS_THREADS];
            s2 += (double)x[i + 2 * LOSS_THREADS];
            s3 += (double)x[i + 3 * LOSS_THREADS];
        }
        for (; i < n; i += LOSS_THREADS) s0 += (double)x[i];
        return (s0 + s1) + (s2 + s3);
    };
    xa = sum4(da + (size_t)t * Na, Na);
    if (beta != 0.0) xb = sum4(db + (size_t)t * Nb, Nb);
    sa[threadIdx.x] = xa;
    sb[threadIdx.x] = xb;
    __syncthreads();
    for (int h = LOSS_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sa[threadIdx.x] += sa[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double w = p.frame_w ? (double)p.frame_w[t] : 1.0;
        p.loss[t] = w * (alpha * sa[0] + beta * sb[0]);
    }
}

__global__ __launch_bounds__(LOSS_THREADS) void k_loss(LossParams p) { loss_body(p, grid_blk()); }

// ---------------------------------------------------------------- one pass, both directions
constexpr int BD_THREADS = 256;
constexpr int BD_TILE = 256;   // targets staged in LDS per step, one per thread
constexpr int BD_SUB = 64;     // the rows' sub-tile, as in k_nn_exact
constexpr int BD_BLK = 16;     // targets per column block, reduced inside the wave
constexpr int BD_CPITCH = BD_BLK + 4;  // a lane's column values of one block, padded
// lane l's values start at l * BD_CPITCH + (l / 16) * 8, so the 64 lanes of one step of the
// transposed scan (16 targets x 4 quarters of the wave) spread evenly over the banks
constexpr int BD_CBUF = 64 * BD_CPITCH + 3 * 8;  // floats per wave

struct BidirParams {
    const float *A;  // rows [T,Na,3]
    const float *B;  // targets [T,Nb,3]
    int32_t *idx_a;  // row results, or slice partials [S][T][Na] when the targets are sliced
    float *dist_a;
    unsigned long long *colkey;  // [T][row blocks][Nb]: (distance bits << 32) | global lane
    size_t slice_stride;         // T * Na with slices, 0 without
    int Na, Nb, slice_len;
};

// logical workgroup: x = row block, y = frame, z = target slice
template <int QPT>
__device__ __forceinline__ void bidir_body(const BidirParams &pr, const Blk &blk) {
    const float *__restrict__ A = pr.A;
    const float *__restrict__ B = pr.B;
    const int Na = pr.Na, Nb = pr.Nb;
    __shared__ float4 tile[2][BD_TILE];
    __shared__ __align__(16) float colbuf[4][BD_CBUF];
    __shared__ unsigned long long colres[2][BD_TILE];
    const int t = blk.y, wg = blk.x, nwg = blk.gx;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float *At = A + (size_t)t * Na * 3;
    const float *Bt = B + (size_t)t * Nb * 3;
    const int j_begin = blk.z * pr.slice_len;
    const int j_end = min(Nb, j_begin + pr.slice_len);
    const int glane = wg * BD_THREADS + (int)threadIdx.x;  // lanes in row order over the frame
    const int r0 = glane * QPT;
    const float nan = __builtin_nanf("");
    const unsigned long long none = ~0ull;
    // rows past Na are NaN: their distances never win a minimum in either direction
    float qx[QPT], qy[QPT], qz[QPT], best[QPT];
    int bsub[QPT];
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
        const bool ok = r0 + k < Na;
        const float *q = At + 3 * (size_t)(ok ? r0 + k : 0);
        qx[k] = ok ? q[0] : nan;
        qy[k] = ok ? q[1] : nan;
        qz[k] = ok ? q[2] : nan;
        best[k] = __builtin_inff();
        bsub[k] = j_begin;
    }
    // the transposed scan of a block: lane (quarter qd, target jt) reads the 16 lanes 16 qd ..
    float *mycol = &colbuf[wave][lane * BD_CPITCH + (lane >> 4) * 8];
    const int jt = lane & (BD_BLK - 1), qd = lane >> 4;
    const float *rdcol = &colbuf[wave][16 * qd * BD_CPITCH + qd * 8 + jt];
    unsigned long long *keyrow = pr.colkey + ((size_t)t * nwg + wg) * Nb;
    auto load_target = [&](int j) {
        if (j < j_end) {
            const float *p = Bt + 3 * (size_t)j;
            return make_float4(p[0], p[1], p[2], 0.f);
        }
        return make_float4(nan, nan, nan, 0.f);  // padding targets: NaN distances
    };
    const int ntiles = (j_end - j_begin + BD_TILE - 1) / BD_TILE;
    colres[0][threadIdx.x] = none;
    colres[1][threadIdx.x] = none;
    tile[0][threadIdx.x] = load_target(j_begin + (int)threadIdx.x);
    float4 nxt = make_float4(nan, nan, nan, 0.f);
    if (ntiles > 1) nxt = load_target(j_begin + BD_TILE + (int)threadIdx.x);
    __syncthreads();
    for (int it = 0; it < ntiles; ++it) {
        const int base = j_begin + it * BD_TILE;
        const int n = min(BD_TILE, j_end - base);
        const int buf = it & 1;
        const float4 *tl = tile[buf];
        for (int s0 = 0; s0 < n; s0 += BD_SUB) {
            float m[QPT];
#pragma unroll
            for (int k = 0; k < QPT; ++k) m[k] = __builtin_inff();
#pragma unroll 1
            for (int b0 = s0; b0 < s0 + BD_SUB; b0 += BD_BLK) {
                // two groups of four targets per iteration (a full unroll spills registers)
#pragma unroll 2
                for (int jj = 0; jj < BD_BLK; jj += 4) {
                    const float4 p0 = tl[b0 + jj], p1 = tl[b0 + jj + 1];
                    const float4 p2 = tl[b0 + jj + 2], p3 = tl[b0 + jj + 3];
                    float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
#pragma unroll
                    for (int k = 0; k < QPT; ++k) {
                        const float d0 = canon_d2(qx[k], qy[k], qz[k], p0.x, p0.y, p0.z);
                        const float d1 = canon_d2(qx[k], qy[k], qz[k], p1.x, p1.y, p1.z);
                        const float d2 = canon_d2(qx[k], qy[k], qz[k], p2.x, p2.y, p2.z);
                        const float d3 = canon_d2(qx[k], qy[k], qz[k], p3.x, p3.y, p3.z);
                        m[k] = __builtin_fminf(__builtin_fminf(m[k], d0), d1);
                        m[k] = __builtin_fminf(__builtin_fminf(m[k], d2), d3);
                        c0 = k ? __builtin_fminf(c0, d0) : d0;
                        c1 = k ? __builtin_fminf(c1, d1) : d1;
                        c2 = k ? __builtin_fminf(c2, d2) : d2;
                        c3 = k ? __builtin_fminf(c3, d3) : d3;
                    }
                    *reinterpret_cast<float4 *>(mycol + jj) = make_float4(c0, c1, c2, c3);
                }
                // the wave reads its own block back transposed (a wave's LDS accesses take
                // effect in program order; the fences keep the compiler to it)
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                float v = __builtin_inff();
                int vl = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const float x = rdcol[i * BD_CPITCH];
                    if (x < v) {  // the first lane of the quarter on ties
                        v = x;
                        vl = i;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                unsigned long long key = ((unsigned long long)__float_as_uint(v) << 32) |
                                         (unsigned)(wg * BD_THREADS + wave * 64 + 16 * qd + vl);
                unsigned long long o = __shfl_xor(key, 16, 64);
                key = o < key ? o : key;
                o = __shfl_xor(key, 32, 64);
                key = o < key ? o : key;
                // the workgroup's minimum per target, the first lane in row order on ties
                if (qd == 0) atomicMin(&colres[buf][b0 + jt], key);
            }
            // rows: the first sub-tile with a strictly smaller minimum is remembered
#pragma unroll
            for (int k = 0; k < QPT; ++k)
                if (m[k] < best[k]) {
                    best[k] = m[k];
                    bsub[k] = base + s0;
                }
        }
        // stage the prefetched next tile, prefetch the one after
        if (it + 1 < ntiles) {
            tile[buf ^ 1][threadIdx.x] = nxt;
            if (it + 2 < ntiles) nxt = load_target(base + 2 * BD_TILE + (int)threadIdx.x);
        }
        __syncthreads();  // the tile's column keys are complete; the next tile is staged
        if ((int)threadIdx.x < n) keyrow[base + threadIdx.x] = colres[buf][threadIdx.x];
        colres[buf][threadIdx.x] = none;  // ready for tile it + 2 (after the next barrier)
    }
    // rows: rescan the winning sub-tile for the first exact match
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
        const int r = r0 + k;
        if (r >= Na) continue;
        const int js = bsub[k];
        const int je = min(js + BD_SUB, j_end);
        int found = js;
        for (int j = js; j < je; ++j) {
            const float *p = Bt + 3 * (size_t)j;
            if (canon_d2(qx[k], qy[k], qz[k], p[0], p[1], p[2]) == best[k]) {
                found = j;
                break;
            }
        }
        const size_t o = (size_t)blk.z * pr.slice_stride + (size_t)t * Na + r;
        pr.idx_a[o] = found;
        pr.dist_a[o] = best[k];
    }
}

template <int QPT>
__global__ __launch_bounds__(BD_THREADS, 4) void k_nn_bidir(BidirParams p) {
    bidir_body<QPT>(p, grid_blk_xcd());
}

// Columns: the smallest key over a frame's row blocks gives the minimum and the first lane (in
// row order) reaching it; that lane's rows are evaluated again for the first one whose distance
// equals it.  When no distance is below infinity the result follows k_nn_exact: the first row of
// the first 64-row sub-tile at an infinite distance, or row 0.
struct BidirMergeParams {
    const float *A;
    const float *B;
    const unsigned long long *colkey;
    int32_t *idx_b;
    float *dist_b;
    int Na, Nb, nwg, qpt;
};

constexpr int BM_THREADS = 256;

__device__ __forceinline__ void bidir_merge_body(const BidirMergeParams &pr, const Blk &blk) {
    const int t = blk.y;
    const int j = blk.x * BM_THREADS + (int)threadIdx.x;
    const int Na = pr.Na, Nb = pr.Nb, nwg = pr.nwg;
    if (j >= Nb) return;
    const unsigned long long *kp = pr.colkey + (size_t)t * nwg * Nb + j;
    unsigned long long key = kp[0];
    for (int w = 1; w < nwg; ++w) {
        const unsigned long long o = kp[(size_t)w * Nb];
        key = o < key ? o : key;
    }
    const float v = __uint_as_float((unsigned)(key >> 32));
    const float *At = pr.A + (size_t)t * Na * 3;
    const float *pb = pr.B + ((size_t)t * Nb + j) * 3;
    const float bx = pb[0], by = pb[1], bz = pb[2];
    int first, last;
    if (v < __builtin_inff()) {
        first = (int)(unsigned)key * pr.qpt;
        last = min(first + pr.qpt, Na);
    } else {
        first = 0;
        last = min(BD_SUB, Na);
    }
    int found = first < Na && v < __builtin_inff() ? first : 0;
    for (int i = first; i < last; ++i) {
        const float *a = At + 3 * (size_t)i;
        if (canon_d2(a[0], a[1], a[2], bx, by, bz) == v) {
            found = i;
            break;
        }
    }
    pr.idx_b[(size_t)t * Nb + j] = found;
    pr.dist_b[(size_t)t * Nb + j] = v;
}

__global__ __launch_bounds__(BM_THREADS) void k_bidir_merge(BidirMergeParams p) {
    bidir_merge_body(p, grid_blk_xcd());
}

}  // namespace

// Workgroups of one launch that are resident on the chip at once (occupancy x compute units),
// for the current device; callers keep the answer (the library drives one kind of GPU).
template <class K>
static long resident_blocks(K kern, int threads) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 256;
    }
    return (long)std::max(per_cu, 1) * std::max(cus, 1);
}

// Equal-length workgroups run in whole rounds of `resident`: the number of target slices S (a
// power of two, at most max_s, each slice at least min_len targets) that minimises the time
// ceil(blocks * S / resident) / S; a larger S must gain more than 2%.
static int round_slices(long blocks, long resident, int Np, int min_len, int max_s) {
    int best = 1;
    double best_cost = std::ceil((double)blocks / resident);
    for (int s = 2; s <= max_s && (long)Np / s >= min_len; s *= 2) {
        const double cost = std::ceil((double)blocks * s / resident) / s;
        if (cost < best_cost * 0.98) {
            best_cost = cost;
            best = s;
        }
    }
    return best;
}

// One pass for both directions pays when there are enough row blocks to fill the chip; smaller
// problems use the two searches of k_nn_exact.  The targets are split over S slices (rows merged
// in slice order afterwards, like k_nn_exact's slices) so that the workgroups, all of the same
// length, fill whole rounds of the chip: S minimises ceil(x_S) / S, x_S = workgroups / resident
// workgroups.
struct BidirPlan {
    int qpt = 0, nwg = 0, slices = 1, slice_len = 0;
};

static BidirPlan bidir_plan(int Na, int Nb, int T) {
    BidirPlan p;
    const long wg8 = (long)T * ((Na + BD_THREADS * 8 - 1) / (BD_THREADS * 8));
    const long wg4 = (long)T * ((Na + BD_THREADS * 4 - 1) / (BD_THREADS * 4));
    if (wg8 >= 512)
        p.qpt = 8;
    else if (wg4 >= 256)
        p.qpt = 4;
    else
        return p;
    p.nwg = (Na + BD_THREADS * p.qpt - 1) / (BD_THREADS * p.qpt);
    static const long res8 = resident_blocks(k_nn_bidir<8>, BD_THREADS);
    static const long res4 = resident_blocks(k_nn_bidir<4>, BD_THREADS);
    const long resident = p.qpt == 8 ? res8 : res4;
    const int s = round_slices((long)T * p.nwg, resident, Nb, 2 * BD_TILE, 16);
    // slices are whole tiles; rounding them up may leave fewer slices than asked for
    p.slice_len = ((Nb + s - 1) / s + BD_TILE - 1) / BD_TILE * BD_TILE;
    p.slices = (Nb + p.slice_len - 1) / p.slice_len;
    return p;
}

size_t nn_bidir_scratch_bytes(int T, int Na, int Nb) {
    const BidirPlan p = bidir_plan(Na, Nb, T);
    if (!p.qpt) return 0;
    size_t b = Arena::need((size_t)T * p.nwg * Nb, sizeof(unsigned long long));
    if (p.slices > 1) b += Arena::need((size_t)p.slices * T * Na, 4) * 2;
    return b;
}

bool launch_nn_bidir(const float *A, int Na, const float *B, int Nb, int T, int32_t *idx_a,
                     float *dist_a, int32_t *idx_b, float *dist_b, char *scratch, hipStream_t st) {
    const BidirPlan pl = bidir_plan(Na, Nb, T);
    if (!pl.qpt) return false;
    Arena ar;
    ar.base = scratch;
    ar.cap = nn_bidir_scratch_bytes(T, Na, Nb);
    BidirParams bp;
    bp.A = A;
    bp.B = B;
    bp.colkey = ar.take<unsigned long long>((size_t)T * pl.nwg * Nb);
    bp.idx_a = idx_a;
    bp.dist_a = dist_a;
    bp.slice_stride = 0;
    if (pl.slices > 1) {
        bp.idx_a = ar.take<int32_t>((size_t)pl.slices * T * Na);
        bp.dist_a = ar.take<float>((size_t)pl.slices * T * Na);
        bp.slice_stride = (size_t)T * Na;
    }
    bp.Na = Na;
    bp.Nb = Nb;
    bp.slice_len = pl.slice_len;
    const dim3 grid(pl.nwg, T, pl.slices);
    if (pl.qpt == 8)
        dispatch(KT_BIDIR8, k_nn_bidir<8>, grid, BD_THREADS, bp, st);
    else
        dispatch(KT_BIDIR4, k_nn_bidir<4>, grid, BD_THREADS, bp, st);
    if (pl.slices > 1) {
        const size_t total = (size_t)T * Na;
        NNMergeParams mp;
        mp.pidx = bp.idx_a;
        mp.pdist = bp.dist_a;
        mp.idx = idx_a;
        mp.dist = dist_a;
        mp.qlist = nullptr;
        mp.qcount = nullptr;
        mp.slice_stride = total;
        mp.slices = pl.slices;
        mp.Nq = Na;
        mp.T = T;
        dispatch(KT_NN_MERGE, k_nn_merge,
                 dim3((unsigned)((total + MERGE_THREADS - 1) / MERGE_THREADS)), MERGE_THREADS, mp,
                 st);
    }
    BidirMergeParams mp;
    mp.A = A;
    mp.B = B;
    mp.colkey = bp.colkey;
    mp.idx_b = idx_b;
    mp.dist_b = dist_b;
    mp.Na = Na;
    mp.Nb = Nb;
    mp.nwg = pl.nwg;
    mp.qpt = pl.qpt;
    dispatch(KT_BIDIR_MERGE, k_bidir_merge, dim3((Nb + BM_THREADS - 1) / BM_THREADS, T),
             BM_THREADS, mp, st);
    return true;
}

// target slices of the one-direction search: enough workgroups to fill the chip, in whole rounds
static int nn_slices(int Nq, int Np, int T, int qpt) {
    const long qblocks = (Nq + NN_THREADS * qpt - 1) / (NN_THREADS * qpt);
    const long blocks = qblocks * T;
    static const long res8 = resident_blocks(k_nn_exact<8>, NN_THREADS);
    static const long res4 = resident_blocks(k_nn_exact<4>, NN_THREADS);
    static const long res1 = resident_blocks(k_nn_exact<1>, NN_THREADS);
    const long resident = qpt == 8 ? res8 : qpt == 4 ? res4 : res1;
    return round_slices(blocks, resident, Np, 2 * NN_TILE, 64);
}

static int nn_qpt(int Nq) { return Nq >= 16384 ? 8 : (Nq >= 4096 ? 4 : 1); }

size_t nn_exact_scratch_bytes(int T, int Nq, int Np) {
    const int s = nn_slices(Nq, Np, T, nn_qpt(Nq));
    if (s == 1) return 0;
    return Arena::need((size_t)s * T * Nq, 4) * 2;
}

static void launch_nn_exact_impl(const float *Q, int Nq, const float *P, int Np, int T,
                                 int32_t *idx, float *dist, char *scratch, int qpt, int s,
                                 const int32_t *qlist, const int32_t *qcount, hipStream_t st) {
    const int slice_len = (Np + s - 1) / s;
    const size_t stride = (size_t)T * Nq;
    int32_t *pidx = idx;
    float *pdist = dist;
    if (s > 1) {
        pidx = reinterpret_cast<int32_t *>(scratch);
        pdist = reinterpret_cast<float *>(scratch + Arena::need((size_t)s * T * Nq, 4));
    }
    // without slices the kernel writes final rows itself (slice_stride 0 marks that case)
    const size_t kstride = s > 1 ? stride : 0;
    const int qblocks = (Nq + NN_THREADS * qpt - 1) / (NN_THREADS * qpt);
    const dim3 grid(qlist ? 1 : qblocks, T, s);
    NNParams np;
    np.Q = Q;
    np.P = P;
    np.idx = pidx;
    np.dist = pdist;
    np.qlist = qlist;
    np.qcount = qcount;
    np.slice_stride = kstride;
    np.Nq = Nq;
    np.Np = Np;
    np.slice_len = slice_len;
    if (qpt == 8)
        dispatch(KT_NN8, k_nn_exact<8>, grid, NN_THREADS, np, st);
    else if (qpt == 4)
        dispatch(KT_NN4, k_nn_exact<4>, grid, NN_THREADS, np, st);
    else
        dispatch(KT_NN1, k_nn_exact<1>, grid, NN_THREADS, np, st);
    if (s > 1) {
        const size_t total = (size_t)T * Nq;
        NNMergeParams mp;
        mp.pidx = pidx;
        mp.pdist = pdist;
        mp.idx = idx;
        mp.dist = dist;
        mp.qlist = qlist;
        mp.qcount = qcount;
        mp.slice_stride = stride;
        mp.slices = s;
        mp.Nq = Nq;
        mp.T = T;
        dispatch(KT_NN_MERGE, k_nn_merge, dim3((unsigned)((total + MERGE_THREADS - 1) / MERGE_THREADS)),
                 MERGE_THREADS, mp, st);
    }
}

void launch_nn_exact_ws(const float *Q, int Nq, const float *P, int Np, int T, int32_t *idx,
                        float *dist, char *scratch, hipStream_t st) {
    const int qpt = nn_qpt(Nq);
    launch_nn_exact_impl(Q, Nq, P, Np, T, idx, dist, scratch, qpt, nn_slices(Nq, Np, T, qpt),
                         nullptr, nullptr, st);
}

// slices for a list of unknown length: split the targets so that a short list still spreads
// over several workgroups
static int list_slices(int Np) {
    int s = 1;
    while (s < 16 && (long)Np / (s * 2) >= 4096) s *= 2;
    return s;
}

size_t nn_exact_list_scratch_bytes(int T, int Nq, int Np) {
    const int s = list_slices(Np);
    if (s == 1) return 0;
    return Arena::need((size_t)s * T * Nq, 4) * 2;
}

void launch_nn_exact_list(const float *Q, int Nq, const float *P, int Np, int T,
                          const int32_t *qlist, const int32_t *qcount, int32_t *idx, float *dist,
                          char *scratch, hipStream_t st) {
    launch_nn_exact_impl(Q, Nq, P, Np, T, idx, dist, scratch, 1, list_slices(Np), qlist, qcount,
                         st);
}

void launch_loss(const float *dist_a, const float *dist_b, int T, int Na, int Nb, int reduction,
                 const float *frame_w, double *loss, hipStream_t s) {
    const double alpha = reduction == DC_RED_SIM2REAL_SUM ? 1.0 : 1.0 / (double)Na;
    const double beta = reduction == DC_RED_SIM2REAL_SUM ? 0.0 : 1.0 / (double)Nb;
    LossParams lp;
    lp.da = dist_a;
    lp.db = dist_b;
    lp.frame_w = frame_w;
    lp.loss = loss;
    lp.alpha = alpha;
    lp.beta = beta;
    lp.Na = Na;
    lp.Nb = Nb;
    dispatch(KT_LOSS, k_loss, dim3(T), LOSS_THREADS, lp, s);
}

void register_nn_kernels(BatchedKernel *table) {
    table[KT_NN1] = batched_kernel<NNParams, nn_exact_body<1>, NN_THREADS, 2048>();
    table[KT_NN4] = batched_kernel<NNParams, nn_exact_body<4>, NN_THREADS, 2048>();
    // the eight-queries-per-lane body keeps four waves per SIMD: 1,024 blocks are all resident
    table[KT_NN8] = batched_kernel<NNParams, nn_exact_body<8>, NN_THREADS, 1024>();
    table[KT_NN_MERGE] = batched_kernel<NNMergeParams, nn_merge_body, MERGE_THREADS, 512>();
    table[KT_LOSS] = batched_kernel<LossParams, loss_body, LOSS_THREADS, 256>();
    // four workgroups per compute unit, like the direct kernel
    table[KT_BIDIR8] = batched_kernel<BidirParams, bidir_body<8>, BD_THREADS, 1024, 4>();
    table[KT_BIDIR4] = batched_kernel<BidirParams, bidir_body<4>, BD_THREADS, 1024, 4>();
    table[KT_BIDIR_MERGE] = batched_kernel<BidirMergeParams, bidir_merge_body, BM_THREADS, 1024>();
}

}  // namespace dc
