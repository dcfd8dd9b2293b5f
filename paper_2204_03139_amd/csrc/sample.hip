// Area-weighted surface sampling (arXiv 2204.03139, Sec. III-B, Eq. 3).
//
// Two kernels per call:
//   k_area_cdf   one workgroup per frame: face areas in double (all lanes), then the running sum
//                C_k = C_{k-1} + A_k in double by one wave, equal bit for bit to the left-to-right
//                sum (index stability needs the same rounding as a sequential sum).
//   k_sample     one lane per point: random words (given, or Philox4x64-10), inverse-CDF face
//                choice by an upper-bound binary search, barycentric point in float.
// Built with -ffp-contract=off: only the fma calls written out below are fused.
#include "batch.h"

namespace dc {
namespace {

#ifndef DC_AREA_CDF_THREADS
#define DC_AREA_CDF_THREADS 1024
#endif
constexpr int AC_THREADS = DC_AREA_CDF_THREADS;  // one wave sums, the other waves compute areas
constexpr int AC_CHUNK = 4000;  // faces per chunk (two buffers, padded: 80 KB of LDS)
constexpr int AC_GROUP = 5;     // faces per thread and chunk: 4000 faces over 960 or 1024 threads

__device__ __forceinline__ bool face_ok(const int32_t *fv, int V) {
    const int32_t i0 = fv[0], i1 = fv[1], i2 = fv[2];
    return (unsigned)i0 < (unsigned)V && (unsigned)i1 < (unsigned)V && (unsigned)i2 < (unsigned)V;
}

// |(p2-p1) x (p3-p1)| / 2 with every product and difference rounded in double.
__device__ __forceinline__ double tri_area_f64(const float *p1, const float *p2, const float *p3) {
    const double ax = (double)p2[0] - (double)p1[0];
    const double ay = (double)p2[1] - (double)p1[1];
    const double az = (double)p2[2] - (double)p1[2];
    const double bx = (double)p3[0] - (double)p1[0];
    const double by = (double)p3[1] - (double)p1[1];
    const double bz = (double)p3[2] - (double)p1[2];
    const double nx = ay * bz - az * by;
    const double ny = az * bx - ax * bz;
    const double nz = ax * by - ay * bx;
    const double sq = nx * nx + ny * ny + nz * nz;
    return 0.5 * __builtin_sqrt(sq);
}

// The running sum over one chunk, in place over entries [0, n) of cur, continuing from `run` (the
// sum of the chunks before it), by the 64 lanes of one wave.  The result is the left-to-right
// double sum C_k = C_{k-1} + A_k bit for bit, without its chain of dependent additions:
//   While a partial sum s lies in one binade [2^E, 2^(E+1)), it is an integer multiple m of the
//   spacing u = 2^(E-52) there, and rounding s + A to that grid does not depend on m: with
//   A / u = q + f (q an integer, 0 <= f < 1) the rounded sum is (m + q + [f > 1/2]) u, except
//   when f is exactly 1/2 (the tie goes to the even multiple, which depends on m) or when
//   m + q + [f > 1/2] reaches 2^53 (the sum leaves the binade and the grid changes).
// So the sums over a window of 64 x RS_PER areas are m_0 plus a prefix sum of the integers
// q + [f > 1/2], taken by a wave scan in double: a sum of non-negative integers is exact while it
// is below 2^53 and, rounded, stays at or above 2^53 once it reaches it, whatever the order.  The
// first area of the window that is a tie or leaves the binade (a NaN or infinite area does) is
// added by one lane exactly as in the plain chain, and the next window starts after it; when a
// window stops within its first RS_BURST positions the lane goes on through RS_BURST areas, so ties
// or binade changes in a row cost no more than the plain chain.  A zero sum skips the zero areas
// after it (0 + 0 = 0); a sum that is not finite, or below the normal range, ends the chunk in the
// plain chain.  `cur` is a chunk buffer: entries [n, n + RS_WIN) are padding that a window may
// load, and the 64 slots from AC_CHUNK + RS_WIN on take the stores a window does not want.
constexpr int RS_PER = 15;  // odd: lanes 120 bytes apart read and write on different LDS banks
constexpr int RS_WIN = 64 * RS_PER;
constexpr int RS_BURST = 64;

// the value of lane (l - n) in the same row of 16 lanes, or 0 where that is outside the row
template <int CTRL>
__device__ __forceinline__ double row_shifted(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// the value of lane l - 1 (0 on lane 0)
__device__ __forceinline__ double lane_before(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x138, 0xF, 0xF, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double lane_value(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// sum of v over lanes 0..lane (v: non-negative integers in double)
__device__ __forceinline__ double wave_prefix(double v, int lane) {
    v = v + row_shifted<0x111>(v);  // row_shr:1
    v = v + row_shifted<0x112>(v);  // row_shr:2
    v = v + row_shifted<0x114>(v);  // row_shr:4
    v = v + row_shifted<0x118>(v);  // row_shr:8
    const double r0 = lane_value(v, 15), r1 = lane_value(v, 31), r2 = lane_value(v, 47);
    const double r01 = r0 + r1;
    const int row = lane >> 4;
    if (row == 1) v = v + r0;
    if (row == 2) v = v + r01;
    if (row == 3) v = v + (r01 + r2);
    return v;
}

__device__ __forceinline__ void plain_sum(double *cur, int i0, int i1, double &run) {
    double r = run;
    int i = i0;
    for (; i + 8 <= i1; i += 8) {  // eight loads in flight, then eight dependent additions
        double x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = cur[i + j];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            r = r + x[j];
            cur[i + j] = r;
        }
    }
    for (; i < i1; ++i) {
        r = r + cur[i];
        cur[i] = r;
    }
    run = r;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ void running_sum(double *cur, int n, double &run, int lane) {
    constexpr double LIM = 9007199254740992.0;  // 2^53
    int k = 0;
    while (k < n) {
        const int avail = n - k;
        const double s = run;  // the same on every lane
        const int eb = (int)(((unsigned long long)__double_as_longlong(s) >> 52) & 0x7FF);
        const int base = lane * RS_PER;
        int stop;  // window position where the plain chain takes over
        if (s == 0.0) {
            int first = RS_PER;
#pragma unroll
            for (int i = RS_PER - 1; i >= 0; --i) {
                const double a = cur[k + base + i];  // past the chunk: the buffer's padding
                if (base + i < avail && a != 0.0) first = i;
            }
            const unsigned long long bal = __ballot(first < RS_PER);
            if (!bal) {  // only zero areas here: their entries are already the zero sums
                k += min(RS_WIN, avail);
                continue;
            }
            const int l = __ffsll((long long)bal) - 1;
            stop = l * RS_PER + __builtin_amdgcn_readlane(first, l);
        } else if (eb == 0 || eb == 0x7FF) {  // below the normal range, infinite or NaN
            if (lane == 0) plain_sum(cur, k, n, run);
            run = lane_value(run, 0);
            return;
        } else {
            const int sh = 1075 - eb;                  // the spacing of s's binade is 2^-sh
            const double ms = __builtin_ldexp(s, sh);  // s / u: an integer in [2^52, 2^53)
            double pre[RS_PER];
            int tie = RS_PER;  // the lane's first tie
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < RS_PER; ++i) {
                const double raw = cur[k + base + i];  // past the chunk: the buffer's padding
                const double a = base + i < avail ? raw : 0.0;
                // A / u + 1/2 is exact while A / u < 2^52, and an area whose A / u is larger
                // leaves the binade whatever its rounding: floor gives q + [f >= 1/2], and the
                // sum is exactly an integer when f is exactly 1/2 (a tie, which stops the window,
                // so that it rounds up here does not matter)
                const double y = __builtin_ldexp(a, sh) + 0.5;
                const double d = __builtin_floor(y);
                if (d == y && tie == RS_PER) tie = i;
                acc = acc + d;  // NaN and infinite areas make the sums leave the binade
                pre[i] = acc;
            }
            const double incl = wave_prefix(acc, lane);
            const double ex = lane_before(incl);  // wave_shr:1
            int inside = 0;  // positions whose sum stays in the binade (sums never decrease)
#pragma unroll
            for (int i = 0; i < RS_PER; ++i) {
                pre[i] = ms + (ex + pre[i]);  // m of position i, in units of u
                inside += pre[i] < LIM ? 1 : 0;
            }
            const int first = min(inside, tie);
            const unsigned long long bal = __ballot(first < RS_PER);
            if (bal) {
                const int l = __ffsll((long long)bal) - 1;
                stop = l * RS_PER + __builtin_amdgcn_readlane(first, l);
            } else {
                stop = RS_WIN;
            }
            // entries at or after the stop go to the lane's spare slot instead (no branches)
#pragma unroll
            for (int i = 0; i < RS_PER; ++i)
                cur[base + i < stop ? k + base + i : AC_CHUNK + RS_WIN + lane] =
                    __builtin_ldexp(pre[i], -sh);
            if (stop == RS_WIN && avail >= RS_WIN) {  // the whole window stayed in the binade
                run = __builtin_ldexp(ms + lane_value(incl, 63), -sh);
                k += RS_WIN;
                continue;
            }
            wave_sync_lds();
            if (stop >= avail || stop == RS_WIN) {
                const int done = min(RS_WIN, avail);
                run = cur[k + done - 1];
                k += done;
                continue;
            }
        }
        // the plain chain from window position `stop`
        const int len = min(stop < RS_BURST ? RS_BURST : 1, avail - stop);
        if (lane == 0) {
            double r = stop == 0 ? s : cur[k + stop - 1];
            plain_sum(cur, k + stop, k + stop + len, r);
            run = r;
        }
        run = lane_value(run, 0);
        wave_sync_lds();
        k += stop + len;
    }
    wave_sync_lds();
}

struct AreaCdfParams {
    const float *verts;
    const int32_t *faces;
    const uint8_t *mask;  // optional: nonzero = the face may be drawn (row t at t * mask_stride)
    size_t mask_stride;
    int V, F;
    double *cdf;
    int32_t *lastpos;
    unsigned *status;
};

// Chunks of AC_CHUNK faces are double-buffered in LDS: while wave 0 runs the sum over chunk c
// (and then copies it out), waves 1.. compute the areas of chunk c + 1.
__device__ __forceinline__ void area_cdf_body(const AreaCdfParams &p, const Blk &blk) {
    const float *__restrict__ verts = p.verts;
    const int32_t *__restrict__ faces = p.faces;
    const int V = p.V, F = p.F;
    // areas, then their running sums; a window of padding lets the summing wave load whole
    // windows past the end of a chunk, and 64 spare slots take its unwanted stores
    __shared__ __align__(16) double area[2][AC_CHUNK + RS_WIN + 64];
    __shared__ int bad;
    __shared__ int lastw[AC_THREADS / 64];
    const int t = blk.x;
    const float *vt = verts + (size_t)t * V * 3;
    double *ct = p.cdf + (size_t)t * F;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) bad = 0;
    int last = -1;  // last face with a positive area, per thread, then per workgroup
    // areas of chunk c into buffer c & 1, by the threads [first, AC_THREADS)
    // (a thread's faces of one chunk are loaded together, AC_GROUP at a time, so their index and
    // corner gathers are in flight at once instead of one face after the other)
    auto areas = [&](int c, int first) {
        const int base = c * AC_CHUNK;
        const int n = min(AC_CHUNK, F - base);
        double *dst = area[c & 1];
        const int stride = AC_THREADS - first;
        for (int k0 = (int)threadIdx.x - first; k0 < n; k0 += AC_GROUP * stride) {
            int32_t fv[AC_GROUP][3];
#pragma unroll
            for (int g = 0; g < AC_GROUP; ++g) {
                const int k = k0 + g * stride;
                const int32_t *f = faces + 3 * (size_t)(base + min(k, n - 1));
                fv[g][0] = f[0];
                fv[g][1] = f[1];
                fv[g][2] = f[2];
            }
            bool ok[AC_GROUP];
            float q[AC_GROUP][3][3];
            unsigned char keep[AC_GROUP];
#pragma unroll
            for (int g = 0; g < AC_GROUP; ++g) {
                ok[g] = face_ok(fv[g], V);
#pragma unroll
                for (int c3 = 0; c3 < 3; ++c3) {
                    const float *v = vt + 3 * (size_t)(ok[g] ? fv[g][c3] : 0);
                    q[g][c3][0] = v[0];
                    q[g][c3][1] = v[1];
                    q[g][c3][2] = v[2];
                }
                const int k = k0 + g * stride;
                keep[g] = p.mask ? p.mask[(size_t)t * p.mask_stride + base + min(k, n - 1)] : 1;
            }
#pragma unroll
            for (int g = 0; g < AC_GROUP; ++g) {
                const int k = k0 + g * stride;
                if (k >= n) break;
                double a = 0.0;
                if (ok[g]) {
                    a = tri_area_f64(q[g][0], q[g][1], q[g][2]);
                    // a face outside the subset takes part with area 0: it is never drawn
                    if (!keep[g]) a = 0.0;
                } else {
                    bad = 1;
                }
                dst[k] = a;
                last = (a > 0.0) ? base + k : last;
            }
        }
    };
    const int nchunk = (F + AC_CHUNK - 1) / AC_CHUNK;
    __syncthreads();  // `bad` is cleared before any thread may set it
    areas(0, 0);
    __syncthreads();
    double run = 0.0;  // the running sum, held by thread 0
    for (int c = 0; c < nchunk; ++c) {
        const int base = c * AC_CHUNK;
        const int n = min(AC_CHUNK, F - base);
        double *cur = area[c & 1];
        if (wave == 0) {
            running_sum(cur, n, run, lane);
            for (int k = lane; k < n; k += 64) ct[base + k] = cur[k];
        } else if (c + 1 < nchunk) {
            areas(c + 1, 64);
        }
        __syncthreads();
    }
    // faces are visited in increasing order per thread, so the maximum is the last positive one
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) last = max(last, __shfl_xor(last, off, 64));
    if (lane == 0) lastw[wave] = last;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < AC_THREADS / 64; ++w) last = max(last, lastw[w]);
        const bool degenerate = !(run > 0.0) || !__builtin_isfinite(run);
        p.lastpos[t] = (degenerate || bad) ? -1 : last;
        if (bad) atomicOr(p.status, (unsigned)ST_BAD_FACE);
        if (degenerate) atomicOr(p.status, (unsigned)ST_DEGENERATE);
    }
}

__global__ __launch_bounds__(AC_THREADS) void k_area_cdf(AreaCdfParams p) {
    area_cdf_body(p, grid_blk());
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64->128 products
// with a Weyl key schedule.
struct Words4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox_words(uint64_t seed, uint32_t t, uint32_t i) {
    uint64_t c0 = i, c1 = t, c2 = 0, c3 = 0;
    uint64_t k0 = seed, k1 = 0;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
        const uint64_t p0hi = __umul64hi(m0, c0), p0lo = m0 * c0;
        const uint64_t p1hi = __umul64hi(m1, c2), p1lo = m1 * c2;
        const uint64_t n0 = p1hi ^ c1 ^ k0;
        const uint64_t n2 = p0hi ^ c3 ^ k1;
        c0 = n0;
        c1 = p1lo;
        c2 = n2;
        c3 = p0lo;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    Words4 w;
    w.w0 = (uint32_t)c0;
    w.w1 = (uint32_t)(c0 >> 32);
    w.w2 = (uint32_t)(c1 >> 32);
    w.w3 = (uint32_t)(c2 >> 32);
    return w;
}

constexpr int SP_THREADS = 256;

struct SampleParams {
    const float *verts;
    const int32_t *faces;
    int V, F, N;
    uint64_t seed;
    const uint32_t *uniforms;
    const double *cdf;
    const int32_t *lastpos;
    float *points;
    int32_t *face_idx;
    float *bary;
};

__device__ __forceinline__ void sample_body(const SampleParams &pr, const Blk &blk) {
    const float *__restrict__ verts = pr.verts;
    const int32_t *__restrict__ faces = pr.faces;
    const int V = pr.V, F = pr.F, N = pr.N;
    const uint32_t *__restrict__ uniforms = pr.uniforms;
    const double *__restrict__ cdf = pr.cdf;
    float *__restrict__ points = pr.points;
    int32_t *__restrict__ face_idx = pr.face_idx;
    float *__restrict__ bary = pr.bary;
    const int t = blk.y;
    const int i = blk.x * SP_THREADS + threadIdx.x;
    if (i >= N) return;
    const size_t o = (size_t)t * N + i;
    const int lp = pr.lastpos[t];
    if (lp < 0) {  // degenerate frame or bad faces: reported through the status word
        const float nan = __builtin_nanf("");
        points[3 * o] = nan;
        points[3 * o + 1] = nan;
        points[3 * o + 2] = nan;
        bary[3 * o] = 0.f;
        bary[3 * o + 1] = 0.f;
        bary[3 * o + 2] = 0.f;
        face_idx[o] = -1;
        return;
    }
    Words4 w;
    if (uniforms) {
        const uint4 u = reinterpret_cast<const uint4 *>(uniforms)[o];
        w.w0 = u.x;
        w.w1 = u.y;
        w.w2 = u.z;
        w.w3 = u.w;
    } else {
        w = philox_words(pr.seed, (uint32_t)t, (uint32_t)i);
    }
    // inverse CDF: first k with C_k > r * S
    const double *ct = cdf + (size_t)t * F;
    const uint64_t bits = (((uint64_t)w.w1 << 32) | (uint64_t)w.w0) >> 11;
    const double r = (double)bits * 0x1p-53;
    const double target = r * ct[F - 1];
    int lo = 0, hi = F;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ct[mid] > target)
            hi = mid;
        else
            lo = mid + 1;
    }
    const int f = (lo < F) ? lo : lp;
    // barycentric point, Eq. 3, with the square-root weights
    const float r1 = (float)(w.w2 >> 8) * 0x1p-24f;
    const float r2 = (float)(w.w3 >> 8) * 0x1p-24f;
    const float s = __builtin_sqrtf(r1);
    const float bu = 1.0f - s;
    const float bv = s * (1.0f - r2);
    const float bw = s * r2;
    const int32_t *fv = faces + 3 * (size_t)f;
    const float *vt = verts + (size_t)t * V * 3;
    const float *p1 = vt + 3 * (size_t)fv[0];
    const float *p2 = vt + 3 * (size_t)fv[1];
    const float *p3 = vt + 3 * (size_t)fv[2];
    // the three corners are read whole (one 12-byte load each) before any store
    float c1[3], c2[3], c3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c1[k] = p1[k];
        c2[k] = p2[k];
        c3[k] = p3[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        points[3 * o + k] = __builtin_fmaf(bw, c3[k], __builtin_fmaf(bv, c2[k], bu * c1[k]));
    bary[3 * o] = bu;
    bary[3 * o + 1] = bv;
    bary[3 * o + 2] = bw;
    face_idx[o] = f;
}

__global__ __launch_bounds__(SP_THREADS) void k_sample(SampleParams p) { sample_body(p, grid_blk_xcd()); }

}  // namespace

size_t sample_scratch_bytes(int T, int F) {
    return Arena::need((size_t)T * F, sizeof(double)) + Arena::need((size_t)T, sizeof(int32_t));
}

void launch_area_cdf(const float *verts, const int32_t *faces, int T, int V, int F,
                     const uint8_t *mask, int mask_per_frame, double *cdf, int32_t *lastpos,
                     unsigned *status, hipStream_t s) {
    AreaCdfParams ap;
    ap.verts = verts;
    ap.faces = faces;
    ap.mask = mask;
    ap.mask_stride = mask_per_frame ? (size_t)F : 0;
    ap.V = V;
    ap.F = F;
    ap.cdf = cdf;
    ap.lastpos = lastpos;
    ap.status = status;
    dispatch(KT_AREA_CDF, k_area_cdf, dim3(T), AC_THREADS, ap, s);
}

void launch_sample(const float *verts, const int32_t *faces, int T, int V, int F, int N,
                   uint64_t seed, const uint32_t *uniforms, const uint8_t *mask, int mask_per_frame,
                   float *points, int32_t *face_idx, float *bary, double *cdf_scratch,
                   int32_t *lastpos_scratch, unsigned *status, hipStream_t s) {
    launch_area_cdf(verts, faces, T, V, F, mask, mask_per_frame, cdf_scratch, lastpos_scratch,
                    status, s);
    SampleParams sp;
    sp.verts = verts;
    sp.faces = faces;
    sp.V = V;
    sp.F = F;
    sp.N = N;
    sp.seed = seed;
    sp.uniforms = uniforms;
    sp.cdf = cdf_scratch;
    sp.lastpos = lastpos_scratch;
    sp.points = points;
    sp.face_idx = face_idx;
    sp.bary = bary;
    dispatch(KT_SAMPLE, k_sample, dim3((N + SP_THREADS - 1) / SP_THREADS, T), SP_THREADS, sp, s);
}

void register_sample_kernels(BatchedKernel *table) {
    table[KT_AREA_CDF] = batched_kernel<AreaCdfParams, area_cdf_body, AC_THREADS, 256>();
    table[KT_SAMPLE] = batched_kernel<SampleParams, sample_body, SP_THREADS, 1024>();
}

}  // namespace dc
