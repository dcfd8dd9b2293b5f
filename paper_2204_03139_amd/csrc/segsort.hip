// Stable, atomic-free sort of per-frame integer keys (LSD radix, 8-bit digits).
//
// One workgroup of 1024 lanes (16 waves of 64) sorts one frame.  Items are visited in chunks of
// 1024 in index order.  Inside a wave, lanes holding the same digit are found with eight ballots;
// a lane's rank is the number of lower lanes in its group, and the group's lowest lane writes the
// group size into a per-wave histogram in LDS (distinct digits, so no two writers collide).  A
// prefix over (wave, digit) then gives every item its output slot, preserving input order among
// equal digits.  Two sweeps per digit (count, then scatter), no atomics, so the permutation is
// the same on every run.  The sorted keys and the original positions are the outputs.
#include "dc_internal.h"

namespace dc {
namespace {

constexpr int SS_THREADS = 1024;
constexpr int SS_WAVES = SS_THREADS / 64;
constexpr int SS_BINS = 256;

__device__ __forceinline__ int load_key(const int32_t *keys, size_t o, int limit) {
    const int k = keys[o];
    return (k < 0 || k > limit) ? limit : k;
}

__global__ __launch_bounds__(SS_THREADS) void k_segsort(const int32_t *__restrict__ keys, int N,
                                                        int key_limit, int passes,
                                                        int32_t *__restrict__ tk0,
                                                        int32_t *__restrict__ tv0,
                                                        int32_t *__restrict__ tk1,
                                                        int32_t *__restrict__ tv1,
                                                        int32_t *__restrict__ out_keys,
                                                        int32_t *__restrict__ out_vals) {
    __shared__ int whist[SS_WAVES][SS_BINS];
    __shared__ int running[SS_BINS];
    const int t = blockIdx.x;
    const size_t fo = (size_t)t * N;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const int32_t *sk = (p == 0) ? nullptr : ((p & 1) ? tk0 : tk1);
        const int32_t *sv = (p == 0) ? nullptr : ((p & 1) ? tv0 : tv1);
        int32_t *dk = (p == passes - 1) ? out_keys : ((p & 1) ? tk1 : tk0);
        int32_t *dv = (p == passes - 1) ? out_vals : ((p & 1) ? tv1 : tv0);

        // ---- count sweep: digit totals
        if (threadIdx.x < SS_BINS) running[threadIdx.x] = 0;
        for (int c = 0; c < N; c += SS_THREADS) {
            for (int k = threadIdx.x; k < SS_WAVES * SS_BINS; k += SS_THREADS)
                (&whist[0][0])[k] = 0;
            __syncthreads();
            const int e = c + threadIdx.x;
            const bool valid = e < N;
            int key = 0;
            if (valid) key = sk ? sk[fo + e] : load_key(keys, fo + e, key_limit);
            const int d = (key >> shift) & (SS_BINS - 1);
            unsigned long long m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1;
                const unsigned long long bb = __ballot(valid && bit);
                m &= bit ? bb : ~bb;
            }
            if (valid && __popcll(m & below) == 0) whist[wave][d] = __popcll(m);
            __syncthreads();
            if (threadIdx.x < SS_BINS) {
                int acc = running[threadIdx.x];
                for (int w = 0; w < SS_WAVES; ++w) acc += whist[w][threadIdx.x];
                running[threadIdx.x] = acc;
            }
            __syncthreads();
        }
        // exclusive prefix over digits
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int b = 0; b < SS_BINS; ++b) {
                const int c = running[b];
                running[b] = acc;
                acc += c;
            }
        }
        __syncthreads();
        // ---- scatter sweep
        for (int c = 0; c < N; c += SS_THREADS) {
            for (int k = threadIdx.x; k < SS_WAVES * SS_BINS; k += SS_THREADS)
                (&whist[0][0])[k] = 0;
            __syncthreads();
            const int e = c + threadIdx.x;
            const bool valid = e < N;
            int key = 0, val = 0;
            if (valid) {
                key = sk ? sk[fo + e] : load_key(keys, fo + e, key_limit);
                val = sv ? sv[fo + e] : e;
            }
            const int d = (key >> shift) & (SS_BINS - 1);
            unsigned long long m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1;
                const unsigned long long bb = __ballot(valid && bit);
                m &= bit ? bb : ~bb;
            }
            const int rank = __popcll(m & below);
            if (valid && rank == 0) whist[wave][d] = __popcll(m);
            __syncthreads();
            if (threadIdx.x < SS_BINS) {  // per digit: offsets of each wave's group
                int acc = running[threadIdx.x];
                for (int w = 0; w < SS_WAVES; ++w) {
                    const int c2 = whist[w][threadIdx.x];
                    whist[w][threadIdx.x] = acc;
                    acc += c2;
                }
                running[threadIdx.x] = acc;
            }
            __syncthreads();
            if (valid) {
                const int pos = whist[wave][d] + rank;
                dk[fo + pos] = key;
                dv[fo + pos] = val;
            }
            __syncthreads();
        }
    }
}

}  // namespace

static int ss_passes(int key_limit) {
    int bits = 1;
    while (bits < 31 && (1 << bits) <= key_limit) ++bits;
    return (bits + 7) / 8;
}

size_t segsort_scratch_bytes(int T, int N) { return 4 * Arena::need((size_t)T * N, 4); }

void launch_segsort(const int32_t *keys, int T, int N, int key_limit, int32_t *out_keys,
                    int32_t *out_vals, char *scratch, hipStream_t s) {
    const size_t piece = Arena::need((size_t)T * N, 4);
    int32_t *tk0 = reinterpret_cast<int32_t *>(scratch);
    int32_t *tv0 = reinterpret_cast<int32_t *>(scratch + piece);
    int32_t *tk1 = reinterpret_cast<int32_t *>(scratch + 2 * piece);
    int32_t *tv1 = reinterpret_cast<int32_t *>(scratch + 3 * piece);
    hipLaunchKernelGGL(k_segsort, dim3(T), dim3(SS_THREADS), 0, s, keys, N, key_limit,
                       ss_passes(key_limit), tk0, tv0, tk1, tv1, out_keys, out_vals);
}

}  // namespace dc
