// Area-weighted surface sampling (arXiv 2204.03139, Sec. III-B, Eq. 3).
//
// Two kernels per call:
//   k_area_cdf   one workgroup per frame: face areas in double (all lanes), then the running sum
//                C_k = C_{k-1} + A_k in double by one lane, in face order, so the CDF is the exact
//                left-to-right sum (index stability needs the same rounding as a sequential sum).
//   k_sample     one lane per point: random words (given, or Philox4x64-10), inverse-CDF face
//                choice by an upper-bound binary search, barycentric point in float.
// Built with -ffp-contract=off: only the fma calls written out below are fused.
#include "batch.h"

namespace dc {
namespace {

#ifndef DC_AREA_CDF_THREADS
#define DC_AREA_CDF_THREADS 1024
#endif
constexpr int AC_THREADS = DC_AREA_CDF_THREADS;  // one lane sums, the other waves compute areas
constexpr int AC_CHUNK = 4000;  // faces per chunk: two chunk buffers of doubles stay under 64 KiB

__device__ __forceinline__ bool face_ok(const int32_t *fv, int V) {
    const int32_t i0 = fv[0], i1 = fv[1], i2 = fv[2];  // one 12-byte load
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

// Chunks of AC_CHUNK faces are double-buffered in LDS: while one lane of wave 0 runs the
// sequential sum over chunk c (and wave 0 then copies it out), waves 1.. compute the areas of
// chunk c + 1, so the area gathers hide behind the dependent chain of additions.
__device__ __forceinline__ void area_cdf_body(const AreaCdfParams &p, const Blk &blk) {
    const float *__restrict__ verts = p.verts;
    const int32_t *__restrict__ faces = p.faces;
    const int V = p.V, F = p.F;
    // areas, then their running sums; 16 entries of padding take the chain's read-ahead
    __shared__ __align__(16) double area[2][AC_CHUNK + 16];
    __shared__ int bad;
    __shared__ int lastw[AC_THREADS / 64];
    const int t = blk.x;
    const float *vt = verts + (size_t)t * V * 3;
    double *ct = p.cdf + (size_t)t * F;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) bad = 0;
    int last = -1;  // last face with a positive area, per thread, then per workgroup
    // areas of chunk c into buffer c & 1, by the threads [first, AC_THREADS)
    auto areas = [&](int c, int first) {
        const int base = c * AC_CHUNK;
        const int n = min(AC_CHUNK, F - base);
        double *dst = area[c & 1];
        for (int k = (int)threadIdx.x - first; k < n; k += AC_THREADS - first) {
            const int32_t *fv = faces + 3 * (size_t)(base + k);
            double a = 0.0;
            if (face_ok(fv, V)) {
                a = tri_area_f64(vt + 3 * (size_t)fv[0], vt + 3 * (size_t)fv[1],
                                 vt + 3 * (size_t)fv[2]);
                // a face outside the subset takes part with area 0: it is never drawn
                if (p.mask && !p.mask[(size_t)t * p.mask_stride + base + k]) a = 0.0;
            } else {
                bad = 1;
            }
            dst[k] = a;
            last = (a > 0.0) ? base + k : last;
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
            if (lane == 0) {  // the sequential sum, in face order
                // groups of 8 areas in two register sets: the next group's loads are in flight
                // while this group's additions run, so the chain waits on the additions only
                // (the last read-ahead ends at most 8 entries past the chunk, in the padding)
                double2 *c2 = reinterpret_cast<double2 *>(cur);
                const int n16 = n & ~15;
                double2 ga[4], gb[4];
                auto load = [&](double2 (&x)[4], int k) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) x[i] = c2[k / 2 + i];
                };
                auto sum = [&](double2 (&x)[4], int k) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        run = run + x[i].x;
                        x[i].x = run;
                        run = run + x[i].y;
                        x[i].y = run;
                        c2[k / 2 + i] = x[i];
                    }
                };
                load(ga, 0);
                for (int k = 0; k < n16; k += 16) {
                    load(gb, k + 8);
                    sum(ga, k);
                    load(ga, k + 16);
                    sum(gb, k + 8);
                }
                for (int k = n16; k < n; ++k) {
                    run = run + cur[k];
                    cur[k] = run;
                }
            }
            // lane 0's sums are visible to the rest of its wave once the wave reconverges
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

void launch_sample(const float *verts, const int32_t *faces, int T, int V, int F, int N,
                   uint64_t seed, const uint32_t *uniforms, const uint8_t *mask, int mask_per_frame,
                   float *points, int32_t *face_idx, float *bary, double *cdf_scratch,
                   int32_t *lastpos_scratch, unsigned *status, hipStream_t s) {
    AreaCdfParams ap;
    ap.verts = verts;
    ap.faces = faces;
    ap.mask = mask;
    ap.mask_stride = mask_per_frame ? (size_t)F : 0;
    ap.V = V;
    ap.F = F;
    ap.cdf = cdf_scratch;
    ap.lastpos = lastpos_scratch;
    ap.status = status;
    dispatch(KT_AREA_CDF, k_area_cdf, dim3(T), AC_THREADS, ap, s);
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
