// Stable, atomic-free sort of per-frame integer keys (LSD radix, 8-bit digits).
//
// Each digit pass is three launches over blocks of 1024 items (many blocks per frame; a frame
// small enough for one workgroup's LDS is sorted in one launch instead, see k_ss_small):
//   k_ss_hist    each block counts its digits: within a wave, lanes holding the same digit are
//                found with eight ballots, the group's lowest lane records the group size in a
//                per-wave LDS row (distinct digits, so no two writers collide); the block sums the
//                rows and stores counts[t][digit][block];
//   k_ss_scan    one workgroup per frame turns the counts, in (digit, block) order, into
//                exclusive offsets;
//   k_ss_scatter each block ranks its items again the same way, in item order (four rounds of 256
//                items, waves in order inside a round), and writes item e to
//                offset[digit][block] + rank, which preserves the input order among equal keys.
// No atomics anywhere, so the permutation is the same on every run.  Keys outside [0, limit] are
// clamped to limit (they sort last); with `mark_invalid` such an item also carries the complement
// of its position (a negative value), so that a key range of exactly 2^k valid keys needs k bits.
#include "batch.h"

namespace dc {
namespace {

constexpr int SB_THREADS = 256;
constexpr int SB_WAVES = SB_THREADS / 64;
constexpr int SB_ROUNDS = 4;
constexpr int SB_ITEMS = SB_THREADS * SB_ROUNDS;  // items per block
constexpr int BINS = 256;

// lanes of this wave whose `valid` item has the same digit as this lane
__device__ __forceinline__ unsigned long long same_digit(bool valid, int d) {
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1;
        const unsigned long long bb = __ballot(valid && bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

struct SortIO {
    const int32_t *src_keys;  // previous pass output, or nullptr for the first pass
    const int32_t *src_vals;
    const int32_t *keys;      // first pass input
    int limit;
    int mark_invalid;         // first pass: an out-of-range key's value is ~position
};

__device__ __forceinline__ void read_item(const SortIO &io, size_t o, int e, int &key, int &val) {
    if (io.src_keys) {
        key = io.src_keys[o];
        val = io.src_vals[o];
        return;
    }
    const int k = io.keys[o];
    const bool bad = k < 0 || k > io.limit;
    key = bad ? io.limit : k;
    val = (bad && io.mark_invalid) ? ~e : e;
}

struct SortPassParams {
    SortIO io;
    int32_t *counts;  // per (frame, digit, block) counts, then their exclusive offsets
    int32_t *dst_keys;
    int32_t *dst_vals;
    int N, shift, nblk;
};

__device__ __forceinline__ void ss_hist_body(const SortPassParams &pr, const Blk &b) {
    const SortIO io = pr.io;
    const int N = pr.N, shift = pr.shift, nblk = pr.nblk;
    int32_t *__restrict__ counts = pr.counts;
    __shared__ int whist[SB_WAVES][BINS];
    __shared__ int total[BINS];
    const int t = b.y, blk = b.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    total[threadIdx.x] = 0;
    for (int r = 0; r < SB_ROUNDS; ++r) {
        for (int k = threadIdx.x; k < SB_WAVES * BINS; k += SB_THREADS) (&whist[0][0])[k] = 0;
        __syncthreads();
        const int e = blk * SB_ITEMS + r * SB_THREADS + threadIdx.x;
        const bool valid = e < N;
        int key = 0, val = 0;
        if (valid) read_item(io, (size_t)t * N + e, e, key, val);
        const int d = (key >> shift) & (BINS - 1);
        const unsigned long long m = same_digit(valid, d);
        if (valid && __popcll(m & below) == 0) whist[wave][d] = __popcll(m);
        __syncthreads();
        int acc = total[threadIdx.x];
        for (int w = 0; w < SB_WAVES; ++w) acc += whist[w][threadIdx.x];
        total[threadIdx.x] = acc;
        __syncthreads();
    }
    counts[((size_t)t * BINS + threadIdx.x) * nblk + blk] = total[threadIdx.x];
}

__global__ __launch_bounds__(SB_THREADS) void k_ss_hist(SortPassParams p) {
    ss_hist_body(p, grid_blk_xcd());
}

// exclusive prefix over (digit, block) of one frame, in place: each thread sums a contiguous run
// (a multiple of four entries, read and written as 16-byte vectors whose loads are issued
// together), the runs' totals are scanned across the workgroup (in-wave shuffles, then the 16 wave
// totals), and each thread rewrites its run from its exclusive start.  The counts of a frame start
// at a multiple of 256 entries, so the vectors are aligned.
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_UNROLL = 4;  // 16-byte vectors per batch of loads
__device__ __forceinline__ void ss_scan_body(const SortPassParams &pr, const Blk &b) {
    __shared__ int wsum[SCAN_THREADS / 64];
    const int nblk = pr.nblk;
    const int t = b.x;
    int32_t *c = pr.counts + (size_t)t * BINS * nblk;
    const int n = BINS * nblk;  // a multiple of 256, so of 4
    const int per = ((n + SCAN_THREADS - 1) / SCAN_THREADS + 3) & ~3;
    const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int4 *c4 = reinterpret_cast<int4 *>(c);
    const int lo4 = lo / 4, hi4 = hi / 4;  // lo and hi are multiples of 4
    int s = 0;
    for (int k = lo4; k < hi4; k += SCAN_UNROLL) {
        int4 v[SCAN_UNROLL];
#pragma unroll
        for (int u = 0; u < SCAN_UNROLL; ++u) v[u] = (k + u < hi4) ? c4[k + u] : make_int4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < SCAN_UNROLL; ++u) s += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    int incl = s;  // inclusive scan of the run totals inside the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    int acc = before + incl - s;
    for (int k = lo4; k < hi4; k += SCAN_UNROLL) {
        int4 v[SCAN_UNROLL];
#pragma unroll
        for (int u = 0; u < SCAN_UNROLL; ++u) v[u] = (k + u < hi4) ? c4[k + u] : make_int4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < SCAN_UNROLL; ++u) {
            if (k + u >= hi4) break;
            int4 o;
            o.x = acc;
            acc += v[u].x;
            o.y = acc;
            acc += v[u].y;
            o.z = acc;
            acc += v[u].z;
            o.w = acc;
            acc += v[u].w;
            c4[k + u] = o;
        }
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_ss_scan(SortPassParams p) {
    ss_scan_body(p, grid_blk());
}

__device__ __forceinline__ void ss_scatter_body(const SortPassParams &pr, const Blk &b) {
    const SortIO io = pr.io;
    const int N = pr.N, shift = pr.shift, nblk = pr.nblk;
    const int32_t *__restrict__ offsets = pr.counts;
    int32_t *__restrict__ dst_keys = pr.dst_keys;
    int32_t *__restrict__ dst_vals = pr.dst_vals;
    __shared__ int whist[SB_WAVES][BINS];
    __shared__ int running[BINS];
    const int t = b.y, blk = b.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    running[threadIdx.x] = offsets[((size_t)t * BINS + threadIdx.x) * nblk + blk];
    for (int r = 0; r < SB_ROUNDS; ++r) {
        for (int k = threadIdx.x; k < SB_WAVES * BINS; k += SB_THREADS) (&whist[0][0])[k] = 0;
        __syncthreads();
        const int e = blk * SB_ITEMS + r * SB_THREADS + threadIdx.x;
        const bool valid = e < N;
        int key = 0, val = 0;
        if (valid) read_item(io, (size_t)t * N + e, e, key, val);
        const int d = (key >> shift) & (BINS - 1);
        const unsigned long long m = same_digit(valid, d);
        const int rank = __popcll(m & below);
        if (valid && rank == 0) whist[wave][d] = __popcll(m);
        __syncthreads();
        {  // per digit: starting slot of each wave's group in this round
            int acc = running[threadIdx.x];
            for (int w = 0; w < SB_WAVES; ++w) {
                const int c = whist[w][threadIdx.x];
                whist[w][threadIdx.x] = acc;
                acc += c;
            }
            running[threadIdx.x] = acc;
        }
        __syncthreads();
        if (valid) {
            const size_t pos = (size_t)t * N + whist[wave][d] + rank;
            dst_keys[pos] = key;
            dst_vals[pos] = val;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(SB_THREADS) void k_ss_scatter(SortPassParams p) {
    ss_scatter_body(p, grid_blk_xcd());
}

static_assert(SB_THREADS == BINS, "one thread per digit bin");

// A segment of at most SM_MAX items whose keys need at most two digit passes is sorted by one
// workgroup in LDS (k_ss_small), in place of the six launches of two passes.  The segment is
// loaded once, every item packed into one word (its 16-bit key, its 14-bit position and a flag for
// an out-of-range key whose value is the complement of the position), and the passes move the words
// between two LDS buffers; the last one writes keys and values out.  Wave w takes the items
// [w P, (w + 1) P) of a pass, P a multiple of 64, in rounds of 64 (item w P + 64 r + lane), so
// (wave, round, lane) is the item order.  Each pass counts the digits per wave (the same
// eight-ballot grouping as above), turns the counts into offsets in (digit, wave) order, and writes
// each item to its wave's running offset for its digit plus its rank among the earlier lanes of
// its round with the same digit: equal keys keep their order.
constexpr int SM_THREADS = 1024;
constexpr int SM_WAVES = SM_THREADS / 64;
// items: two buffers of one word each, 32 KB of LDS.  One workgroup takes about 0.8 us per round
// of its 16 waves (the ballots dominate), so past about 4,096 items the launches of the block
// passes, spread over the chip, are as fast or faster.
constexpr int SM_MAX = 4096;

struct SortSmallParams {
    SortIO io;  // the input keys (src_keys unused)
    int32_t *dst_keys;
    int32_t *dst_vals;
    int N, passes;
};

__device__ __forceinline__ void ss_small_body(const SortSmallParams &pr, const Blk &b) {
    __shared__ unsigned buf[2][SM_MAX];
    __shared__ int wcnt[SM_WAVES][BINS];
    __shared__ int dsum[BINS / 64];
    const int t = b.x;
    const int N = pr.N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int per = (N + SM_THREADS - 1) / SM_THREADS * 64;  // items per wave
    const int rounds = per / 64;
    const int w0 = wave * per;
    // key << 16 | flag << 14 | position (keys are below 2^16 when two passes suffice)
    for (int e = threadIdx.x; e < N; e += SM_THREADS) {
        int key, val;
        read_item(pr.io, (size_t)t * N + e, e, key, val);
        buf[0][e] = ((unsigned)key << 16) | (val < 0 ? 1u << 14 : 0u) | (unsigned)e;
    }
    for (int p = 0; p < pr.passes; ++p) {
        const unsigned *src = buf[p & 1];
        unsigned *dst = buf[(p + 1) & 1];
        const int shift = 16 + 8 * p;
        const bool last = p == pr.passes - 1;
        for (int k = threadIdx.x; k < SM_WAVES * BINS; k += SM_THREADS) (&wcnt[0][0])[k] = 0;
        __syncthreads();
        for (int r = 0; r < rounds; ++r) {
            const int e = w0 + 64 * r + lane;
            const bool valid = e < N;
            const int d = valid ? (int)(src[e] >> shift) & (BINS - 1) : 0;
            const unsigned long long m = same_digit(valid, d);
            if (valid && __popcll(m & below) == 0) wcnt[wave][d] += __popcll(m);
        }
        __syncthreads();
        // offsets in (digit, wave) order: the digit totals scanned by threads 0..255, then each
        // digit's waves in order
        int s = 0, incl = 0;
        if (threadIdx.x < BINS) {
            for (int w = 0; w < SM_WAVES; ++w) s += wcnt[w][threadIdx.x];
            incl = s;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int o = __shfl_up(incl, off, 64);
                if (lane >= off) incl += o;
            }
            if (lane == 63) dsum[wave] = incl;
        }
        __syncthreads();
        if (threadIdx.x < BINS) {
            int base = incl - s;
            for (int w = 0; w < wave; ++w) base += dsum[w];
            for (int w = 0; w < SM_WAVES; ++w) {
                const int c = wcnt[w][threadIdx.x];
                wcnt[w][threadIdx.x] = base;
                base += c;
            }
        }
        __syncthreads();
        for (int r = 0; r < rounds; ++r) {
            const int e = w0 + 64 * r + lane;
            const bool valid = e < N;
            const unsigned word = valid ? src[e] : 0u;
            const int d = (int)(word >> shift) & (BINS - 1);
            const unsigned long long m = same_digit(valid, d);
            const int rank = __popcll(m & below);
            const int pos = wcnt[wave][d] + rank;
            if (valid && rank == 0) wcnt[wave][d] = pos + __popcll(m);
            if (valid) {
                if (last) {
                    const int pe = (int)(word & 0x3FFFu);
                    pr.dst_keys[(size_t)t * N + pos] = (int)(word >> 16);
                    pr.dst_vals[(size_t)t * N + pos] = (word & (1u << 14)) ? ~pe : pe;
                } else {
                    dst[pos] = word;
                }
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(SM_THREADS) void k_ss_small(SortSmallParams p) {
    ss_small_body(p, grid_blk());
}

}  // namespace

static int ss_passes(int key_limit) {
    int bits = 1;
    while (bits < 31 && (1 << bits) <= key_limit) ++bits;
    return (bits + 7) / 8;
}

static int ss_blocks(int N) { return (N + SB_ITEMS - 1) / SB_ITEMS; }

size_t segsort_scratch_bytes(int T, int N) {
    return 4 * Arena::need((size_t)T * N, 4) + Arena::need((size_t)T * BINS * ss_blocks(N), 4);
}

void launch_segsort(const int32_t *keys, int T, int N, int key_limit, int32_t *out_keys,
                    int32_t *out_vals, char *scratch, hipStream_t s, bool mark_invalid) {
    const size_t piece = Arena::need((size_t)T * N, 4);
    int32_t *tk[2] = {reinterpret_cast<int32_t *>(scratch),
                      reinterpret_cast<int32_t *>(scratch + 2 * piece)};
    int32_t *tv[2] = {reinterpret_cast<int32_t *>(scratch + piece),
                      reinterpret_cast<int32_t *>(scratch + 3 * piece)};
    int32_t *counts = reinterpret_cast<int32_t *>(scratch + 4 * piece);
    if (T <= 0 || N <= 0) return;
    const int nblk = ss_blocks(N);
    const int passes = ss_passes(key_limit);
    if (N <= SM_MAX && passes <= 2) {  // one workgroup per segment, in LDS
        SortSmallParams sp;
        sp.io.keys = keys;
        sp.io.src_keys = nullptr;
        sp.io.src_vals = nullptr;
        sp.io.limit = key_limit;
        sp.io.mark_invalid = mark_invalid ? 1 : 0;
        sp.dst_keys = out_keys;
        sp.dst_vals = out_vals;
        sp.N = N;
        sp.passes = passes;
        dispatch(KT_SS_SMALL, k_ss_small, dim3(T), SM_THREADS, sp, s);
        return;
    }
    const dim3 grid(nblk, T);
    for (int p = 0; p < passes; ++p) {
        SortIO io;
        io.keys = keys;
        io.limit = key_limit;
        io.mark_invalid = mark_invalid ? 1 : 0;
        io.src_keys = p == 0 ? nullptr : tk[(p - 1) & 1];
        io.src_vals = p == 0 ? nullptr : tv[(p - 1) & 1];
        int32_t *dk = (p == passes - 1) ? out_keys : tk[p & 1];
        int32_t *dv = (p == passes - 1) ? out_vals : tv[p & 1];
        SortPassParams sp;
        sp.io = io;
        sp.counts = counts;
        sp.dst_keys = dk;
        sp.dst_vals = dv;
        sp.N = N;
        sp.shift = 8 * p;
        sp.nblk = nblk;
        dispatch(KT_SS_HIST, k_ss_hist, grid, SB_THREADS, sp, s);
        dispatch(KT_SS_SCAN, k_ss_scan, dim3(T), SCAN_THREADS, sp, s);
        dispatch(KT_SS_SCATTER, k_ss_scatter, grid, SB_THREADS, sp, s);
    }
}

void register_sort_kernels(BatchedKernel *table) {
    table[KT_SS_HIST] = batched_kernel<SortPassParams, ss_hist_body, SB_THREADS, 1024>();
    table[KT_SS_SCAN] = batched_kernel<SortPassParams, ss_scan_body, SCAN_THREADS, 256>();
    table[KT_SS_SCATTER] = batched_kernel<SortPassParams, ss_scatter_body, SB_THREADS, 1024>();
    table[KT_SS_SMALL] = batched_kernel<SortSmallParams, ss_small_body, SM_THREADS, 256>();
}

}  // namespace dc
