// bf16 matrix-core screen + certified exact refine for the all-pairs nearest neighbours of
// Sec. III-A (Eq. 1/2), in both directions at once: the same indices as the exact single-precision
// search, found faster.
//
// Screen (k_screen): the squared distance is expanded as s_ij = |a_i|^2 + |b_j|^2 - 2 a_i.b_j and
// evaluated as one K=32 dot product per pair on v_mfma_f32_16x16x32_bf16 with fp32 accumulation.
// Each float coordinate is split exactly into three bf16 parts (x = h + m + l); the products
// hH, hM, mH, hL, lH, mM per coordinate (18 K-slots) plus the two norms in three parts each (6
// K-slots) fill 24 of the 32 K-slots, so the matrix unit produces the whole screened distance.
// Rows a stay in registers (16-row tiles: eight per wave); the
// b operands (packed once per frame) stream through a double-buffered LDS stage.  Every 16x16
// result tile feeds both directions with v_min3 only:
//   rows (a -> b): each (lane, row) folds its column of every tile into a running minimum;
//     targets are laid out so that, inside each chunk of SC_CHUNK, result column c holds a
//     contiguous run of SC_RUN targets (a "slot group"); the kernel keeps the two best slot
//     groups and the third-best value per (lane, row);
//   columns (b -> a): each lane folds its 16 rows of a tile into one value per b_j; a lane swap
//     pairs lane groups g and g + 2 (32 rows: a "row group"), and after the next stage's
//     barrier the workgroup reduces its 8 row groups per b_j in LDS and writes the workgroup's
//     minimum, the winning row group and an "ambiguous" flag (a second group within the
//     certificate margin) to a per-workgroup partial array.
// Certificate: every bf16 split is exact and every bf16 product is exact in fp32, so
// |s_ij - d_ij| <= C (|a_i|^2 + |b_j|^2) (at most 24 fp32 roundings at 2^-23 on a sum of absolute
// products <= 2.02 (|a|^2+|b|^2), plus dropped split products and float norms).  The canonical
// float distance fma(dz,dz,fma(dy,dy,dx*dx)) is within 5u of the exact one (u = 2^-24).  Hence
// any index whose canonical distance can equal the minimum has s <= m + Delta(m), m the screened
// minimum of the query, Delta bounding the error at the screened and the canonical winner (both
// within sqrt(m + e) of the query, which bounds their norms).  Candidates pass that test; a query
// with too many candidates or a non-finite minimum is "heavy" and is searched exhaustively.
// Refine: teams of 16 lanes evaluate the canonical distance over the candidates and keep the
// lexicographic (distance, index) minimum: exactly the argmin of the exhaustive search with the
// smallest-index rule.
#include "batch.h"

namespace dc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// tiling (overridable at build time for tuning sweeps)
#ifndef DC_SCREEN_ATILES
#define DC_SCREEN_ATILES 8
#endif
#ifndef DC_SCREEN_STAGE
#define DC_SCREEN_STAGE 256
#endif
#ifndef DC_SCREEN_CHUNK
#define DC_SCREEN_CHUNK 2048
#endif
constexpr int SC_WAVES = 4;
constexpr int SC_THREADS = 64 * SC_WAVES;
#ifndef DC_SCREEN_ATILES_COLS
#define DC_SCREEN_ATILES_COLS 8
#endif
// 16-row query tiles per wave: eight in both screens, at two workgroups per compute unit (232
// registers for one direction, 255 for both; fewer tiles measured slower in both, and the
// two-direction screen amortises its per-stage column reduction over them)
template <bool COLS>
constexpr int sc_atiles() { return COLS ? DC_SCREEN_ATILES_COLS : DC_SCREEN_ATILES; }
template <bool COLS>
constexpr int sc_rows() { return SC_WAVES * sc_atiles<COLS>() * 16; }  // query rows per workgroup
constexpr int SC_STAGE = DC_SCREEN_STAGE;                // targets staged in LDS per step
constexpr int SC_CHUNK = DC_SCREEN_CHUNK;                // targets per tracking chunk
constexpr int SC_TPS = SC_STAGE / 16;                    // tiles per stage
constexpr int SC_RUN = SC_CHUNK / 16;                    // contiguous targets of a slot group
constexpr int SC_PER_THREAD = SC_STAGE / SC_THREADS;     // targets staged per thread
constexpr int SC_ROWPAD = 17;                            // LDS entries per staged tile
static_assert(SC_STAGE % SC_THREADS == 0 && SC_CHUNK % SC_STAGE == 0, "tiling");
constexpr int MAXC = 14;                                 // candidate slot groups per row
constexpr int REC_INTS = 2 + MAXC;                       // n, spare, entries

// bound constant C of the screen error: 24 accumulations at 2^-23 relative on a sum of absolute
// products <= 2.02 (|q|^2 + |p|^2), plus the dropped split products and the float norms
constexpr float SCREEN_C = 6.5e-6f;
constexpr float SCREEN_TAU = 1e-30f;       // absolute slack (denormal flushing of tiny products)
constexpr float CANON_U13 = 13.0f * 5.9604645e-8f;  // 13 u, u = 2^-24

struct Split3 {
    __bf16 h, m, l;
};

// exact three-way split of a float into bf16 parts (round to nearest even at each step)
__device__ __forceinline__ Split3 split3(float x) {
    Split3 s;
    s.h = (__bf16)x;
    const float r1 = x - (float)s.h;
    s.m = (__bf16)r1;
    s.l = (__bf16)(r1 - (float)s.m);
    return s;
}

__device__ __forceinline__ float norm2(float x, float y, float z) {
    return __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x));
}

// K-slot vectors.  Query side: per coordinate [h,h,m,h,l,m], then |q|^2 parts, then ones.
// Target side (of -2p): per coordinate [h,m,h,l,h,m], then ones, then |p|^2 parts.
__device__ __forceinline__ void query_vector(float x, float y, float z, __bf16 (&v)[32]) {
    const float c[3] = {x, y, z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const Split3 s = split3(c[k]);
        v[6 * k + 0] = s.h;
        v[6 * k + 1] = s.h;
        v[6 * k + 2] = s.m;
        v[6 * k + 3] = s.h;
        v[6 * k + 4] = s.l;
        v[6 * k + 5] = s.m;
    }
    const Split3 n = split3(norm2(x, y, z));
    v[18] = n.h;
    v[19] = n.m;
    v[20] = n.l;
    v[21] = (__bf16)1.0f;
    v[22] = (__bf16)1.0f;
    v[23] = (__bf16)1.0f;
#pragma unroll
    for (int k = 24; k < 32; ++k) v[k] = (__bf16)0.0f;
}

__device__ __forceinline__ void target_vector(float x, float y, float z, bool valid,
                                              __bf16 (&v)[32]) {
    const float c[3] = {-2.0f * x, -2.0f * y, -2.0f * z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const Split3 s = split3(valid ? c[k] : 0.0f);
        v[6 * k + 0] = s.h;
        v[6 * k + 1] = s.m;
        v[6 * k + 2] = s.h;
        v[6 * k + 3] = s.l;
        v[6 * k + 4] = s.h;
        v[6 * k + 5] = s.m;
    }
    v[18] = (__bf16)1.0f;
    v[19] = (__bf16)1.0f;
    v[20] = (__bf16)1.0f;
    const Split3 n = split3(valid ? norm2(x, y, z) : 1e30f);  // padding: a huge distance
    v[21] = n.h;
    v[22] = n.m;
    v[23] = n.l;
#pragma unroll
    for (int k = 24; k < 32; ++k) v[k] = (__bf16)0.0f;
}

__device__ __forceinline__ bf16x8 pick8(const __bf16 (&v)[32], int g) {
    bf16x8 r;
    if (g == 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) r[e] = v[e];
    } else if (g == 1) {
#pragma unroll
        for (int e = 0; e < 8; ++e) r[e] = v[8 + e];
    } else if (g == 2) {
#pragma unroll
        for (int e = 0; e < 8; ++e) r[e] = v[16 + e];
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) r[e] = v[24 + e];
    }
    return r;
}

// Target operands of every frame, packed once: target j's three non-zero K-chunks (48 bytes).
// Padding targets up to a whole chunk get a huge norm so they never win a minimum.

// largest squared norm of each frame's targets (for the certificate)
struct NormMaxParams {
    const float *P;
    float *out;
    int32_t *heavy_cnt;
    int Np;
};

constexpr int NM_THREADS = 1024;

__device__ __forceinline__ void norm_max_body(const NormMaxParams &pr, const Blk &blk) {
    const float *__restrict__ P = pr.P;
    const int Np = pr.Np;
    float *__restrict__ out = pr.out;
    int32_t *__restrict__ heavy_cnt = pr.heavy_cnt;
    __shared__ float red[NM_THREADS / 64];
    const int t = blk.x;
    if (threadIdx.x == 0) heavy_cnt[t] = 0;
    const float *pt = P + (size_t)t * Np * 3;
    // four points per step, each read whole (one 12-byte load), their loads in flight together;
    // the maximum does not depend on the order (fmaxf drops NaN whatever the order)
    float m = 0.f;
    int j = threadIdx.x;
    for (; j + 3 * NM_THREADS < Np; j += 4 * NM_THREADS) {
        float c[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float *q = pt + 3 * (size_t)(j + u * NM_THREADS);
            c[u][0] = q[0];
            c[u][1] = q[1];
            c[u][2] = q[2];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) m = fmaxf(m, norm2(c[u][0], c[u][1], c[u][2]));
    }
    for (; j < Np; j += NM_THREADS)
        m = fmaxf(m, norm2(pt[3 * (size_t)j], pt[3 * (size_t)j + 1], pt[3 * (size_t)j + 2]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NM_THREADS / 64; ++w) m = fmaxf(m, red[w]);
        out[t] = m;
    }
}

__global__ __launch_bounds__(NM_THREADS) void k_norm_max(NormMaxParams p) {
    norm_max_body(p, grid_blk());
}

// Certificate threshold: every index whose canonical float distance can equal the minimum has a
// screened value <= threshold(m, nq, nmax), where m is the query's screened minimum, nq its squared
// norm and nmax the largest squared norm among the points it is compared with.  Increasing in m.
__device__ __forceinline__ float threshold(float m, float nq, float nmax) {
    // v_sqrt_f32 is within 1 ulp; every use below is scaled up by `up`, which covers it
    const float up = 1.0001f;
    const float qn = __builtin_amdgcn_sqrtf(nq) * up;
    const float mp = fmaxf(m, 0.f);
    const float e0 = (SCREEN_C * (nq + nmax) + SCREEN_TAU) * up;
    const float r0 = qn + __builtin_amdgcn_sqrtf(mp + e0) * up;
    const float e1 = (SCREEN_C * (nq + r0 * r0) + SCREEN_TAU) * up;  // at the screened winner
    const float d1 = (mp + e1) * (1.0f + CANON_U13) * up;
    const float r1 = qn + __builtin_amdgcn_sqrtf(d1) * up;
    const float e2 = (SCREEN_C * (nq + r1 * r1) + SCREEN_TAU) * up;  // at the canonical winner
    const float th = m + e1 + e2 + CANON_U13 * (mp + e1);
    return th + fabsf(th) * 1e-4f + SCREEN_TAU;
}

// A larger bound that is affine in max(m, 0), for the per-stage ambiguity test of the column
// direction: replacing the squared radii of the threshold above by (a + b)^2 <= 1.125 a^2 + 9 b^2
// makes every term linear, so th(m) <= m + A(nq, nmax) + AFF_B * max(m, 0), with A depending only
// on the point (computed once per target) and AFF_B a constant.  Both carry a 1e-3 relative margin
// for the float evaluation; the margin also exceeds the rounding of the final additions, since a
// negative m is at most the error at the screened winner, which A contains.
constexpr double AFF_C = (double)SCREEN_C, AFF_U13 = 13.0 * 5.9604644775390625e-8;
constexpr float AFF_B = (float)((9 * AFF_C + 9 * AFF_C * (1 + AFF_U13) * (1 + 9 * AFF_C) +
                                 AFF_U13 * (1 + 9 * AFF_C)) * 1.001);

__device__ __forceinline__ float affine_slack(float nq, float nmax) {
    const float e0 = SCREEN_C * (nq + nmax) + SCREEN_TAU;
    const float c1 = SCREEN_C * (2.125f * nq + 9.0f * e0) + SCREEN_TAU;
    const float k = (float)(1.0 + 9 * AFF_C * (1 + AFF_U13) + AFF_U13);
    return (c1 * k + 2.125f * SCREEN_C * nq + SCREEN_TAU) * 1.001f;
}

__device__ __forceinline__ float threshold_affine(float m, float slack) {
    const float th = m + __builtin_fmaf(AFF_B, fmaxf(m, 0.f), slack);
    return th + fabsf(th) * 1e-4f + SCREEN_TAU;
}

// Target operands of every frame, packed once: target j's three non-zero K-chunks (48 bytes), and
// the affine threshold slack of the column direction.  Padding targets up to a whole chunk get a
// huge norm so they never win a minimum.
struct PackParams {
    const float *P;
    const float *nqmax;
    bf16x8 *packed;
    float *slack;
    int Np, Np_pad;
};

__device__ __forceinline__ void pack_body(const PackParams &pr, const Blk &blk) {
    const float *__restrict__ P = pr.P;
    const int Np = pr.Np, Np_pad = pr.Np_pad;
    const int t = blk.y;
    const int j = blk.x * 256 + threadIdx.x;
    if (j >= Np_pad) return;
    const bool valid = j < Np;
    const float *p = P + ((size_t)t * Np + (valid ? j : 0)) * 3;
    const float px = p[0], py = p[1], pz = p[2];  // one 12-byte load (row 0 for padding)
    const float x = valid ? px : 0.f, y = valid ? py : 0.f, z = valid ? pz : 0.f;
    __bf16 v[32];
    target_vector(x, y, z, valid, v);
    bf16x8 *o = pr.packed + ((size_t)t * Np_pad + j) * 3;
    o[0] = pick8(v, 0);
    o[1] = pick8(v, 1);
    o[2] = pick8(v, 2);
    pr.slack[(size_t)t * Np_pad + j] = affine_slack(norm2(x, y, z), pr.nqmax[t]);
}

__global__ __launch_bounds__(256) void k_pack_targets(PackParams p) { pack_body(p, grid_blk()); }

// Column partials are one 16-bit word per (row workgroup, target): a 12-bit code of the
// workgroup's minimum over the target, then the ambiguous flag (bit 3) and the winning row group
// (bits 0-2).  The code is the bf16 pattern of max(v, 0) (the float truncated to 16 bits: rounded
// down) less a per-frame bias, clamped to [0, 4095]: monotone in v, with bf16's 7 mantissa bits
// over 32 binades that end above every squared distance of the frame (at most 4 max|x|^2).  Code 0
// covers everything below the range and negative screened values, code 4095 everything above it.
// Words compare like their codes.
constexpr int PC_MAX = 4095;

// bias of the frame's codes: the top binade of the range is that of 8 max(|a|^2, |b|^2)
__device__ __forceinline__ int part_bias(float nqmax, float npmax) {
    const unsigned et = (__float_as_uint(8.0f * fmaxf(nqmax, npmax)) >> 23) & 0xFFu;
    return et > 31u ? (int)((et - 31u) << 7) : 0;
}

__device__ __forceinline__ int part_code(float v, int bias) {
    const int hb = (int)(__float_as_uint(fmaxf(v, 0.f)) >> 16);
    return min(max(hb - bias, 0), PC_MAX);
}

// a value above everything a code can stand for (infinite for the saturated code)
__device__ __forceinline__ float part_hi(int c, int bias) {
    return c >= PC_MAX ? __builtin_inff() : __uint_as_float((unsigned)(c + 1 + bias) << 16);
}

// the largest word whose code can stand for a value <= th (-1: none; a NaN passes everything)
__device__ __forceinline__ int part_word_limit(float th, int bias) {
    if (th < 0.f) return -1;
    const int c = (th >= 0.f) ? part_code(th, bias) : PC_MAX;
    return (c << 4) | 15;
}

// Column row groups per workgroup: (wave, h), h in {0, 1}, holding the rows 16a + 4g + r of the
// wave with g in {h, h + 2}: lane groups g and g + 2 see the same result columns, and one lane
// swap pairs their partial minima up.
constexpr int SC_GROUPS = SC_WAVES * 2;
constexpr int CP_PAD = SC_TPS + 1;       // column partial buffer: [group][column][tile], padded

// Column partial words of every (row workgroup w, target j) of a frame, laid out in blocks of
// CP_BLOCK targets: [frame][j / CP_BLOCK][w][j % CP_BLOCK].  The merge reads one
// block's rows as one contiguous stream; a screen workgroup's stores stay runs of 16 targets.
constexpr int CP_BLOCK = 128;
static_assert(SC_CHUNK % CP_BLOCK == 0, "padded target counts are whole blocks");
__device__ __forceinline__ size_t part_index(int t, int nwg, int Np_pad, int w, int j) {
    const size_t blk = (size_t)t * (Np_pad / CP_BLOCK) + (size_t)(j / CP_BLOCK);
    return (blk * nwg + w) * CP_BLOCK + (size_t)(j % CP_BLOCK);
}

struct ScreenParams {
    const float *Q;
    const bf16x8 *packed;
    const float *slack;
    const float *npmax;  // per frame: largest squared norm of the targets
    const float *nqmax;  // and of the queries
    int32_t *rec;
    int32_t *heavy_cnt;
    int32_t *heavy_list;
    uint16_t *cpart;
    int Nq, Np, Np_pad;
};

// logical workgroup: x = row block of the frame, y = frame, gx = row blocks per frame
template <bool COLS>
__device__ __forceinline__ void screen_body(const ScreenParams &pr, const Blk &blk) {
    constexpr int ATILES = sc_atiles<COLS>();  // 16-row query tiles per wave
    constexpr int ROWS = sc_rows<COLS>();      // query rows per workgroup
    const float *__restrict__ Q = pr.Q;
    const bf16x8 *__restrict__ packed = pr.packed;
    const float *__restrict__ slack = pr.slack;
    const int Nq = pr.Nq, Np_pad = pr.Np_pad;
    int32_t *__restrict__ rec = pr.rec;
    int32_t *__restrict__ heavy_cnt = pr.heavy_cnt;
    int32_t *__restrict__ heavy_list = pr.heavy_list;
    uint16_t *__restrict__ cpart = pr.cpart;
    // [buffer][K-chunk][entry] -> 16 bytes.  Entry 17*bt + c holds tile bt, result column c: the
    // operand reads (16 columns of one tile) are consecutive and the staging stores (8 tiles of
    // one column, 272 bytes apart) fall in distinct banks; the read address is a per-lane base
    // plus a compile-time offset.  K-chunk 3 is all zeros on the query side and is not stored.
    __shared__ bf16x8 stage[2][3][SC_ROWPAD * SC_TPS];
    // double-buffered by stage parity: the partials of stage s are reduced after the barrier of
    // stage s + 1, so one barrier per stage orders both buffers
    __shared__ float colbuf[COLS ? 2 : 1][COLS ? SC_GROUPS : 1][16][CP_PAD];
    const int nwg = blk.gx, wgx = blk.x, t = blk.y;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;   // K-chunk of the operands; row group of the result
    const int col = lane & 15; // row of the A operand; column (slot) of the result
    const float *Qt = Q + (size_t)t * Nq * 3;
    const bf16x8 *Bt = packed + (size_t)t * Np_pad * 3;
    const int row0 = wgx * ROWS + wave * (ATILES * 16);

    // query operands, held for the whole sweep
    bf16x8 A[ATILES];
#pragma unroll
    for (int a = 0; a < ATILES; ++a) {
        const int r = row0 + 16 * a + col;
        __bf16 v[32];
        if (r < Nq)
            query_vector(Qt[3 * (size_t)r], Qt[3 * (size_t)r + 1], Qt[3 * (size_t)r + 2], v);
        else
            query_vector(0.f, 0.f, 1e15f, v);  // padding row: far from everything
        A[a] = pick8(v, g);
    }

    // per (lane, row): running minimum of the current chunk and the three best chunk minima.  A
    // chunk's minimum carries the chunk's index in its kbits lowest mantissa bits, so the three
    // smallest values travel with their chunks through plain minimum instructions; every value is
    // then within 2^(kbits-22) relative of the minimum it stands for.  The running minimum starts
    // at the largest finite float, so an encoded value is never a NaN.
    const float inf = __builtin_inff();
    const float big = __FLT_MAX__;
    const int nchunk = Np_pad / SC_CHUNK;
    const int kbits = nchunk > 1 ? 32 - __builtin_clz((unsigned)(nchunk - 1)) : 0;
    const unsigned kmask = (1u << kbits) - 1u;
    float m[ATILES][4], b1[ATILES][4], b2[ATILES][4], b3[ATILES][4];
#pragma unroll
    for (int a = 0; a < ATILES; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            m[a][r] = big;
            b1[a][r] = inf;
            b2[a][r] = inf;
            b3[a][r] = inf;
        }
    const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
    const int nstage = Np_pad / SC_STAGE;
    constexpr int SPC = SC_CHUNK / SC_STAGE;  // stages per chunk
    // staging: entry (btl, c) of a stage holds target SC_RUN*c + SC_TPS*(stage in chunk) + btl of
    // its chunk, so result column c of a chunk is the contiguous run [SC_RUN*c, SC_RUN*(c+1))
    int spos[SC_PER_THREAD], soff[SC_PER_THREAD];
#pragma unroll
    for (int u = 0; u < SC_PER_THREAD; ++u) {
        const int e = threadIdx.x + u * SC_THREADS;
        const int c = e / SC_TPS, btl = e % SC_TPS;
        spos[u] = btl * SC_ROWPAD + c;
        soff[u] = SC_RUN * c + btl;
    }
    auto target_of = [&](int st, int u) {
        return (st / SPC) * SC_CHUNK + SC_TPS * (st % SPC) + soff[u];
    };
    // register prefetch of the next stage's operands, double-buffered LDS.  The column threshold
    // slack of the targets a thread stages is prefetched with them and kept until the thread
    // reduces those same targets one stage later (sl_prev: stage st - 1, sl_cur: st, sl_next:
    // st + 1), so the reduction never waits on memory.
    const float *slack_t = slack + (size_t)t * Np_pad;
    float sl_prev[SC_PER_THREAD], sl_cur[SC_PER_THREAD], sl_next[SC_PER_THREAD];
    bf16x8 q[SC_PER_THREAD][3];
#pragma unroll
    for (int u = 0; u < SC_PER_THREAD; ++u) {
        sl_prev[u] = sl_next[u] = 0.f;
        sl_cur[u] = COLS ? slack_t[target_of(0, u)] : 0.f;
        const bf16x8 *src = Bt + (size_t)target_of(0, u) * 3;
        q[u][0] = src[0];
        q[u][1] = src[1];
        q[u][2] = src[2];
    }
    const int gk = (g == 3) ? 0 : g;
    // the column partial offsets of this thread's staged targets in stage 0: a stage's targets
    // lie in one slot group of its chunk, and a slot group lies inside one CP_BLOCK block, so the
    // offset moves by a uniform step from stage to stage
    static_assert(CP_BLOCK % SC_RUN == 0 && SC_CHUNK % CP_BLOCK == 0,
                  "a slot group lies inside one partial block");
    size_t pbase[SC_PER_THREAD];
#pragma unroll
    for (int u = 0; u < SC_PER_THREAD; ++u)
        pbase[u] = COLS ? part_index(t, nwg, Np_pad, wgx, soff[u]) : 0;
    const int pbias = COLS ? part_bias(pr.nqmax[t], pr.npmax[t]) : 0;
    // reduce the workgroup's row groups per target of stage sm and write its partial
    // reduce the workgroup's row groups per target of stage sm and write its partial (padding
    // targets too: the partial arrays span the padded target range)
    auto merge_stage = [&](int sm) {
        const int cb = sm & 1;
#pragma unroll
        for (int u = 0; u < SC_PER_THREAD; ++u) {
            const int e = threadIdx.x + u * SC_THREADS;
            const int c = e / SC_TPS, btl = e % SC_TPS;
            float best = inf, second = inf;
            int bg = 0;
#pragma unroll
            for (int k = 0; k < SC_GROUPS; ++k) {
                const float v = colbuf[COLS ? cb : 0][COLS ? k : 0][c][btl];
                second = __builtin_amdgcn_fmed3f(v, best, second);  // best <= second
                bg = v < best ? k : bg;
                best = fminf(best, v);
            }
            // another row group within the margin of this group's best: the merge must rescan
            // every row of the workgroup for this target
            const float th = threshold_affine(best, sl_prev[u]);
            const bool amb = !(second > th + fabsf(th) * 1e-6f);
            // part_index(t, nwg, Np_pad, wgx, target_of(sm, u)): the thread's chunk-0 offset
            // plus a uniform step
            const size_t o = pbase[u] + (size_t)(sm / SPC) * (SC_CHUNK / CP_BLOCK) * nwg * CP_BLOCK +
                             SC_TPS * (sm % SPC);
            cpart[o] = (uint16_t)(((unsigned)part_code(best, pbias) << 4) | (amb ? 8u : 0u) |
                                  (unsigned)bg);
        }
    };
    for (int st = 0; st < nstage; ++st) {
        const int buf = st & 1;
#pragma unroll
        for (int u = 0; u < SC_PER_THREAD; ++u) {
            stage[buf][0][spos[u]] = q[u][0];
            stage[buf][1][spos[u]] = q[u][1];
            stage[buf][2][spos[u]] = q[u][2];
        }
        if (st + 1 < nstage) {
#pragma unroll
            for (int u = 0; u < SC_PER_THREAD; ++u) {
                if (COLS) sl_next[u] = slack_t[target_of(st + 1, u)];
                const bf16x8 *src = Bt + (size_t)target_of(st + 1, u) * 3;
                q[u][0] = src[0];
                q[u][1] = src[1];
                q[u][2] = src[2];
            }
        }
        __syncthreads();
        if (COLS && st > 0) merge_stage(st - 1);
        // lanes of K-group 3 hold an all-zero query operand, so any finite staged operand gives
        // them zero products: they read K-chunk 0 instead of a stored zero chunk
        const bf16x8 *sb = &stage[buf][gk][col];
        // operands of the next tile pair are read one pair ahead
        bf16x8 N0 = sb[0], N1 = sb[SC_ROWPAD];
#pragma unroll
        for (int bt = 0; bt < SC_TPS; bt += 2) {
            const bf16x8 B0 = N0, B1 = N1;
            if (bt + 2 < SC_TPS) {
                N0 = sb[(bt + 2) * SC_ROWPAD];
                N1 = sb[(bt + 3) * SC_ROWPAD];
            }
            float cm0 = inf, cm1 = inf;
            // issue order, written out: each query tile's two MFMAs go one tile ahead of the
            // minima that read their results, so no minimum waits for the matrix unit (measured
            // faster than the compiler's order, also when it was steered by a one-tile scheduling
            // hint; eight tiles per wave leave no registers for a second tile of lookahead)
            constexpr int LA = 1;
            floatx4 d0[ATILES], d1[ATILES];
#pragma unroll
            for (int a = 0; a < LA; ++a) {
                d0[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a], B0, zero, 0, 0, 0);
                d1[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a], B1, zero, 0, 0, 0);
            }
#pragma unroll
            for (int a = 0; a < ATILES; ++a) {
                if (a + LA < ATILES) {
                    d0[a + LA] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a + LA], B0, zero, 0, 0, 0);
                    d1[a + LA] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a + LA], B1, zero, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) m[a][r] = fminf(fminf(m[a][r], d0[a][r]), d1[a][r]);
                if (COLS) {
                    cm0 = fminf(fminf(cm0, d0[a][0]), d0[a][1]);
                    cm0 = fminf(fminf(cm0, d0[a][2]), d0[a][3]);
                    cm1 = fminf(fminf(cm1, d1[a][0]), d1[a][1]);
                    cm1 = fminf(fminf(cm1, d1[a][2]), d1[a][3]);
                }
            }
            if (COLS) {
                // rows 2-3 of cm0 trade places with rows 0-1 of cm1, so lane group g ends up
                // with the minimum over groups g and g + 2 (mod 4) of tile bt + (g >> 1)
                const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(cm0),
                                                                 __float_as_uint(cm1), false,
                                                                 false);
                const float v = fminf(__uint_as_float(sw[0]), __uint_as_float(sw[1]));
                colbuf[COLS ? (st & 1) : 0][COLS ? wave * 2 + (g & 1) : 0][col][bt + (g >> 1)] = v;
            }
        }
        if ((st + 1) % SPC == 0) {  // end of a tracking chunk
            const unsigned k = (unsigned)(st / SPC);
#pragma unroll
            for (int a = 0; a < ATILES; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float x = __uint_as_float((__float_as_uint(m[a][r]) & ~kmask) | k);
                    b3[a][r] = __builtin_amdgcn_fmed3f(x, b2[a][r], b3[a][r]);
                    b2[a][r] = __builtin_amdgcn_fmed3f(x, b1[a][r], b2[a][r]);
                    b1[a][r] = fminf(x, b1[a][r]);
                    m[a][r] = big;
                }
        }
#pragma unroll
        for (int u = 0; u < SC_PER_THREAD; ++u) {
            sl_prev[u] = sl_cur[u];
            sl_cur[u] = sl_next[u];
        }
    }
    if (COLS) {  // the last stage's partials
        __syncthreads();
        merge_stage(nstage - 1);
    }

    // row certificate and candidate records; the 16 lanes of a group share one row per (a, r).
    // The encoded chunk minima stand for values within a relative kslack of themselves: the
    // certificate is taken at a value above the row's minimum, and a chunk passes when its value
    // does not exceed the threshold widened by the same amount.
    const float npm = pr.npmax[t];
    const float kslack = __uint_as_float((unsigned)(127 + kbits - 21) << 23);  // 2^(kbits-21)
    const unsigned long long gmask = 0xFFFFull << (16 * g);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int a = 0; a < ATILES; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = row0 + 16 * a + 4 * g + r;
            float mi = b1[a][r];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) mi = fminf(mi, __shfl_xor(mi, off, 64));
            float nq = 0.f;
            if (row < Nq)
                nq = norm2(Qt[3 * (size_t)row], Qt[3 * (size_t)row + 1], Qt[3 * (size_t)row + 2]);
            const float theta =
                threshold(mi + fabsf(mi) * kslack + SCREEN_TAU, nq, npm);
            const float thp = theta + fabsf(theta) * kslack + SCREEN_TAU;
            const bool finite = __builtin_isfinite(mi) && __builtin_isfinite(theta) &&
                                __builtin_isfinite(npm);
            const bool k1 = finite && b1[a][r] <= thp;
            const bool k2 = finite && b2[a][r] <= thp;
            const bool over = finite && b3[a][r] <= thp;
            const int c1 = (int)(__float_as_uint(b1[a][r]) & kmask);
            const int c2 = (int)(__float_as_uint(b2[a][r]) & kmask);
            const unsigned long long m1 = __ballot(k1) & gmask;
            const unsigned long long m2 = __ballot(k2) & gmask;
            const unsigned long long mo = __ballot(over) & gmask;
            const int n = __popcll(m1) + __popcll(m2);
            const bool heavy = !finite || n > MAXC || mo != 0ull;
            if (row < Nq) {
                int32_t *rr = rec + ((size_t)t * Nq + row) * REC_INTS;
                if (col == 0) {
                    rr[0] = heavy ? -1 : n;
                    if (heavy) {
                        const int pos = atomicAdd(&heavy_cnt[t], 1);
                        heavy_list[(size_t)t * Nq + pos] = row;
                    }
                }
                if (!heavy) {
                    const int off = __popcll(m1 & below) + __popcll(m2 & below);
                    if (k1) rr[2 + off] = (c1 << 4) | col;
                    if (k2) rr[2 + off + (k1 ? 1 : 0)] = (c2 << 4) | col;
                }
            }
        }
}

// Direct launch, in an XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs, so
// the hardware ids of one XCD are mapped onto one contiguous range of (frame, row block) items and
// each XCD's L2 holds the packed targets of about T/8 frames instead of every frame.  Three
// workgroups per compute unit (at most 168 registers per lane) keep three waves on every SIMD.
template <bool COLS>
__global__ __launch_bounds__(SC_THREADS, sc_atiles<COLS>() <= 4 ? 3 : 2) void k_screen(ScreenParams p) {
    Blk b;
    b.gx = gridDim.x;
    b.gy = gridDim.y;
    b.gz = 1;
    b.z = 0;
    const unsigned total = (unsigned)gridDim.x * gridDim.y;
    const unsigned id = blockIdx.x + (unsigned)gridDim.x * blockIdx.y;
    const unsigned c = id % 8u, k = id / 8u, per = total / 8u, rem = total % 8u;
    const unsigned item = c * per + (c < rem ? c : rem) + k;
    b.y = (int)(item / gridDim.x);
    b.x = (int)(item % gridDim.x);
    screen_body<COLS>(p, b);
}

// Column merge: per target b_j, a running minimum over the workgroup partials and the list of
// workgroups whose partial passed the (affine, never smaller) threshold of the minimum seen so far;
// at the end the list is filtered by the certificate at the final minimum.  Candidates are the
// workgroups passing it; more than CMAXC makes the target heavy.  Record per target: n (or -1 =
// heavy) and up to CMAXC entries (workgroup << 8 | tag), tag = row group | 0x80 if ambiguous.
constexpr int CMAXC = 12;
constexpr int CREC_INTS = 1 + CMAXC + 1;

constexpr int CM_TPT = 2;    // targets per thread: one 32-bit word of two 16-bit partials
#ifndef DC_CM_CAP
#define DC_CM_CAP 16
#endif
#ifndef DC_CM_BATCH
#define DC_CM_BATCH 8
#endif
constexpr int CM_CAP = DC_CM_CAP;      // pending list entries per target, in LDS
constexpr int CM_THREADS = 256;

struct ColmergeParams {
    const float *P;
    const float *slack;  // per-target affine threshold slack (k_pack_targets)
    const uint16_t *cpart;
    const float *nqmax;  // per frame: largest squared norm of the rows (a)
    const float *npmax;  // and of the targets (b)
    int32_t *crec;
    int32_t *heavy_cnt;
    int32_t *heavy_list;
    int Np, Np_pad, nwg;
};

__device__ __forceinline__ void colmerge_body(const ColmergeParams &pr, const Blk &blk) {
    const float *__restrict__ P = pr.P;
    const int Np = pr.Np, Np_pad = pr.Np_pad, nwg = pr.nwg;
    const uint16_t *__restrict__ cpart = pr.cpart;
    int32_t *__restrict__ crec = pr.crec;
    int32_t *__restrict__ heavy_cnt = pr.heavy_cnt;
    int32_t *__restrict__ heavy_list = pr.heavy_list;
    // pending entries (workgroup << 16) | partial word; point counts are at most 2^24, so there
    // are at most 2^16 row workgroups
    __shared__ uint32_t pend[CM_CAP][CM_TPT][CM_THREADS];
    const int t = blk.y;
    const int tid = threadIdx.x;
    const int j0 = (blk.x * CM_THREADS + tid) * CM_TPT;
    if (j0 >= Np) return;
    const float nqm = pr.nqmax[t];
    const int bias = part_bias(nqm, pr.npmax[t]);
    int best[CM_TPT], lim[CM_TPT], cnt[CM_TPT];
    float slk[CM_TPT];
    bool over[CM_TPT];
#pragma unroll
    for (int u = 0; u < CM_TPT; ++u) {
        best[u] = PC_MAX + 1;
        lim[u] = 0x7fffffff;
        cnt[u] = 0;
        over[u] = false;
        slk[u] = pr.slack[(size_t)t * Np_pad + j0 + u];
    }
    // this wave's block of CP_BLOCK targets (CM_TPT per lane): one row of CP_BLOCK partials per
    // row workgroup, the rows consecutive
    const int jb = __builtin_amdgcn_readfirstlane(j0 / CP_BLOCK);  // the same for the whole wave
    const uint16_t *block = cpart + part_index(t, nwg, Np_pad, 0, jb * CP_BLOCK);
    // The partials are taken in batches of CM_BATCH workgroups.  First the batch's smallest word
    // of each target (packed 16-bit minima: words order like their codes) lowers the running
    // minimum and the threshold is recomputed once, at a value above that minimum (the top of its
    // code); then every partial of the batch whose word passes goes on the list.  The threshold
    // only falls, so an entry it excludes at any point is excluded at the end.  A full list drops
    // the entries the current threshold excludes; if none can be dropped the target is made heavy
    // (always correct: it is searched exhaustively).
    auto lower = [&](int u, unsigned mw) {
        best[u] = min(best[u], (int)(mw >> 4));
        lim[u] = part_word_limit(threshold_affine(part_hi(best[u], bias), slk[u]), bias);
    };
    auto append = [&](int u, unsigned word, int w) {
        if ((int)word > lim[u] || over[u]) return;
        if (cnt[u] == CM_CAP) {
            int n = 0;
#pragma unroll 1
            for (int k = 0; k < CM_CAP; ++k) {
                const uint32_t e = pend[k][u][tid];
                if ((int)(e & 0xFFFFu) <= lim[u]) pend[n++][u][tid] = e;
            }
            cnt[u] = n;
            if (n == CM_CAP) {
                over[u] = true;
                return;
            }
        }
        pend[cnt[u]++][u][tid] = ((uint32_t)w << 16) | word;
    };
    typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));
    constexpr int CM_BATCH = DC_CM_BATCH;  // workgroups per batch
    auto merge_batch = [&](const unsigned *v, int nk, int w) {
        ushort2_t m = {(unsigned short)0xFFFFu, (unsigned short)0xFFFFu};
        for (int k = 0; k < nk; ++k) m = __builtin_elementwise_min(m, __builtin_bit_cast(ushort2_t, v[k]));
        lower(0, m.x);
        lower(1, m.y);
        // nothing of the batch passes for either target: the common case, one test per lane
        if ((int)m.x > lim[0] && (int)m.y > lim[1]) return;
        for (int k = 0; k < nk; ++k) {
            append(0, v[k] & 0xFFFFu, w + k);
            append(1, v[k] >> 16, w + k);
        }
    };
    // the next batch's loads in flight while this batch is merged.  Each batch reads through a
    // buffer resource based at its first row, so a load's address is the uniform row offset
    // (scalar) plus the lane's offset: no per-lane 64-bit address math.  The loads are
    // unconditional (the last whole batch re-reads itself, unused), so the waits fall on the
    // batch being merged only.
    static_assert(CP_BLOCK == 64 * CM_TPT, "one wave reads one block");
    const unsigned row_bytes = (unsigned)CP_BLOCK * 2u;
    const unsigned lane_bytes = (unsigned)(j0 % CP_BLOCK) * 2u;
    const int nfull = nwg / CM_BATCH * CM_BATCH;
    auto load_batch = [&](int w0, unsigned (&v)[CM_BATCH]) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(block + (size_t)w0 * CP_BLOCK), 0, (int)(row_bytes * CM_BATCH), 0x00020000);
#pragma unroll
        for (int k = 0; k < CM_BATCH; ++k)
            v[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, lane_bytes, k * row_bytes, 0);
    };
    unsigned nxt[CM_BATCH];
    if (nfull > 0) load_batch(0, nxt);
    int w = 0;
    for (; w < nfull; w += CM_BATCH) {
        unsigned cur[CM_BATCH];
#pragma unroll
        for (int k = 0; k < CM_BATCH; ++k) cur[k] = nxt[k];
        load_batch(w + CM_BATCH < nfull ? w + CM_BATCH : w, nxt);
        merge_batch(cur, CM_BATCH, w);
    }
    if (w < nwg) {  // the last, partial batch
        unsigned cur[CM_BATCH];
        const int nk = nwg - w;
        for (int k = 0; k < nk; ++k)
            cur[k] = *reinterpret_cast<const unsigned *>(block + (size_t)(w + k) * CP_BLOCK + j0 % CP_BLOCK);
        merge_batch(cur, nk, w);
    }
#pragma unroll
    for (int u = 0; u < CM_TPT; ++u) {
        const int j = j0 + u;
        if (j >= Np) break;
        const float *pj = P + ((size_t)t * Np + j) * 3;
        const float np = norm2(pj[0], pj[1], pj[2]);
        // the certificate at a value above the true minimum (the top of the smallest code); a
        // workgroup is kept when the bottom of its code passes it
        const float theta = threshold(part_hi(best[u], bias), np, nqm);
        const bool finite = __builtin_isfinite(theta) && __builtin_isfinite(nqm);
        const int wlim = part_word_limit(theta, bias);
        int32_t *rr = crec + ((size_t)t * Np + j) * CREC_INTS;
        int n = 0;
        if (finite && !over[u]) {
#pragma unroll 1
            for (int k = 0; k < cnt[u]; ++k) {
                const uint32_t e = pend[k][u][tid];
                if ((int)(e & 0xFFFFu) <= wlim) {
                    const int wk = (int)(e >> 16);
                    const int tag = (int)(e & 7u) | ((e & 8u) ? 0x80 : 0);
                    if (n < CMAXC) rr[1 + n] = (wk << 8) | tag;
                    ++n;
                }
            }
        }
        if (!finite || over[u] || n > CMAXC) {
            rr[0] = -1;
            const int pos = atomicAdd(&heavy_cnt[t], 1);
            heavy_list[(size_t)t * Np + pos] = j;
            continue;
        }
        rr[0] = n;
    }
}

__global__ __launch_bounds__(CM_THREADS) void k_colmerge(ColmergeParams p) { colmerge_body(p, grid_blk()); }

__device__ __forceinline__ float canon_d2(float qx, float qy, float qz, const float *p) {
    const float dx = qx - p[0];
    const float dy = qy - p[1];
    const float dz = qz - p[2];
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

constexpr int RF_THREADS = 256;
constexpr int RF_TEAM = 16;                         // lanes per query
constexpr int RF_STEP = 4 * RF_TEAM;                // targets a team covers per step
static_assert(SC_RUN % RF_STEP == 0, "slot groups are whole refine steps");
constexpr int RF_TEAMS = RF_THREADS / RF_TEAM;
constexpr int RF_QUERIES = 256;                     // queries per workgroup (16 per team)

// Every lane keeps the smallest (distance, index) key over the points it evaluates: the distance
// as its float bits in the high word, the point's index in the low word.  A canonical distance is a
// non-negative float or a NaN; non-negative floats order like their bits and every NaN pattern
// orders above +inf, so a NaN never wins.  The initial key is +inf with the largest index, so an
// infinite distance can still win on its index (the smallest index at +inf), as the exhaustive
// search's first-smallest rule gives when no distance is finite.
constexpr unsigned long long RF_NONE = (0x7F800000ull << 32) | 0xFFFFFFFFull;

__device__ __forceinline__ unsigned canon_bits(float qx, float qy, float qz, float px, float py,
                                               float pz) {
    const float dx = qx - px;
    const float dy = qy - py;
    const float dz = qz - pz;
    return __float_as_uint(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
}

// the points i0 .. i0 + 3 (those below Np) of P: their smallest key (the run's minimum and the
// first of its indices that reaches it) folded into `key`
__device__ __forceinline__ void run4_key(unsigned long long &key, float qx, float qy, float qz,
                                         const float *P, int i0, int Np) {
    unsigned d0, d1, d2, d3;
    if (i0 + 3 < Np) {  // a whole run: three 16-byte loads
        const float4 *p4 = reinterpret_cast<const float4 *>(P + 3 * (size_t)i0);
        const float4 u0 = p4[0], u1 = p4[1], u2 = p4[2];
        d0 = canon_bits(qx, qy, qz, u0.x, u0.y, u0.z);
        d1 = canon_bits(qx, qy, qz, u0.w, u1.x, u1.y);
        d2 = canon_bits(qx, qy, qz, u1.z, u1.w, u2.x);
        d3 = canon_bits(qx, qy, qz, u2.y, u2.z, u2.w);
    } else {  // the end of the point array
        const float *p = P + 3 * (size_t)i0;
        d0 = i0 < Np ? canon_bits(qx, qy, qz, p[0], p[1], p[2]) : 0xFFFFFFFFu;
        d1 = i0 + 1 < Np ? canon_bits(qx, qy, qz, p[3], p[4], p[5]) : 0xFFFFFFFFu;
        d2 = i0 + 2 < Np ? canon_bits(qx, qy, qz, p[6], p[7], p[8]) : 0xFFFFFFFFu;
        d3 = 0xFFFFFFFFu;
    }
    const unsigned m = min(min(d0, d1), min(d2, d3));
    const int first = d0 == m ? 0 : (d1 == m ? 1 : (d2 == m ? 2 : 3));
    const unsigned long long k = ((unsigned long long)m << 32) | (unsigned)(i0 + first);
    key = k < key ? k : key;
}

// the smallest key over the 16 lanes of a team (a row of the wave for DPP): rotations by 8, 4, 2
// and 1 lanes within the row.  Returns false when no key beat the initial one (every candidate
// distance a NaN).
template <int CTRL>
__device__ __forceinline__ unsigned long long row_rotated(unsigned long long k) {
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)k, CTRL, 0xF, 0xF, false);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(k >> 32), CTRL, 0xF, 0xF, false);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ bool team_result(unsigned long long key, int &idx, float &dist) {
    static_assert(RF_TEAM == 16, "a team is one DPP row");
    unsigned long long o;
    o = row_rotated<0x128>(key);  // row_ror:8
    key = o < key ? o : key;
    o = row_rotated<0x124>(key);  // row_ror:4
    key = o < key ? o : key;
    o = row_rotated<0x122>(key);  // row_ror:2
    key = o < key ? o : key;
    o = row_rotated<0x121>(key);  // row_ror:1
    key = o < key ? o : key;
    idx = (int)(unsigned)key;
    dist = __uint_as_float((unsigned)(key >> 32));
    return key != RF_NONE;
}

__device__ __forceinline__ void flush_stats(unsigned *cnt, unsigned long long *stats, int live,
                                            unsigned my_cand, unsigned my_heavy, int tl) {
    if (!stats) return;
    if (tl == 0) {
        atomicAdd(&cnt[0], my_cand);
        atomicAdd(&cnt[1], my_heavy);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *slot =
            stats + (size_t)((blockIdx.x + gridDim.x * blockIdx.y) % STATS_SLOTS) * STATS_SLOT_WORDS;
        atomicAdd(&slot[0], (unsigned long long)live);
        atomicAdd(&slot[1], (unsigned long long)cnt[0]);
        atomicAdd(&slot[2], (unsigned long long)cnt[1]);
    }
}

// The workgroup's query records and query points, staged in LDS with coalesced loads issued
// together: the teams then meet global memory only for the points they compare against.
template <int INTS>
__device__ __forceinline__ void stage_queries(const int32_t *rec, const float *Q, int t, int Nq,
                                              int i0, int32_t *srec, float *sq) {
    const int nq = min(RF_QUERIES, Nq - i0);
    const int32_t *rb = rec + ((size_t)t * Nq + i0) * INTS;
    const float *qb = Q + ((size_t)t * Nq + i0) * 3;
#pragma unroll
    for (int u = 0; u < RF_QUERIES * INTS / RF_THREADS; ++u) {
        const int k = threadIdx.x + u * RF_THREADS;
        if (k < nq * INTS) srec[k] = rb[k];
    }
#pragma unroll
    for (int u = 0; u < RF_QUERIES * 3 / RF_THREADS; ++u) {
        const int k = threadIdx.x + u * RF_THREADS;
        if (k < nq * 3) sq[k] = qb[k];
    }
}

// The order in which the teams take the workgroup's queries: sorted by candidate count (a counting
// sort in LDS), so the four teams of a wave, which loop together, get queries of equal count and
// no lane idles through another team's longer list.  Each query's result does not depend on the
// order (heavy queries, count -1, and the slots past the last query sort first).
constexpr int RF_BINS = 16;  // counts -2 .. 13 and above
static_assert(RF_QUERIES == RF_THREADS, "one staged query per thread");
template <int INTS>
__device__ __forceinline__ void order_queries(const int32_t *srec, int nq, int *bins,
                                              int16_t *order) {
    const int q = threadIdx.x;
    const int n = q < nq ? srec[q * INTS] : -2;
    const int key = min(n + 2, RF_BINS - 1);
    if (q < RF_BINS) bins[q] = 0;
    __syncthreads();
    atomicAdd(&bins[key], 1);
    __syncthreads();
    if (q == 0) {
        int sum = 0;
        for (int k = 0; k < RF_BINS; ++k) {
            const int c = bins[k];
            bins[k] = sum;
            sum += c;
        }
    }
    __syncthreads();
    order[atomicAdd(&bins[key], 1)] = (int16_t)q;
    __syncthreads();
}

// Row refine (a -> b): candidate slot groups of light rows; heavy rows are left to the exact
// kernel.  A team of 16 lanes takes one query; each 64-target step gives every lane one run of 4
// consecutive targets (48 contiguous bytes).
struct RefineParams {
    const float *Q;  // queries (rows a for the row refine, targets b for the column refine)
    const float *P;  // points searched (b, or a)
    const int32_t *rec;
    int32_t *idx;
    float *dist;
    unsigned long long *stats;
    int Nq, Np;
};

__device__ __forceinline__ void refine_body(const RefineParams &pr, const Blk &blk) {
    const float *__restrict__ Q = pr.Q;
    const float *__restrict__ P = pr.P;
    const int Nq = pr.Nq, Np = pr.Np;
    const int32_t *__restrict__ rec = pr.rec;
    int32_t *__restrict__ idx = pr.idx;
    float *__restrict__ dist = pr.dist;
    unsigned long long *__restrict__ stats = pr.stats;
    __shared__ unsigned cnt[2];
    __shared__ int32_t srec[RF_QUERIES * REC_INTS];
    __shared__ float sq[RF_QUERIES * 3];
    const int t = blk.y;
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __shared__ int bins[RF_BINS];
    __shared__ int16_t order[RF_QUERIES];
    stage_queries<REC_INTS>(rec, Q, t, Nq, blk.x * RF_QUERIES, srec, sq);
    __syncthreads();
    order_queries<REC_INTS>(srec, min(RF_QUERIES, Nq - blk.x * RF_QUERIES), bins, order);
    const int team = threadIdx.x / RF_TEAM, tl = threadIdx.x % RF_TEAM;
    const float *Pt = P + (size_t)t * Np * 3;
    unsigned my_cand = 0, my_heavy = 0;
    for (int qq = 0; qq < RF_QUERIES / RF_TEAMS; ++qq) {
        const int li = order[qq * RF_TEAMS + team];
        const int i = blk.x * RF_QUERIES + li;
        const int32_t *rr = srec + li * REC_INTS;
        const int n = (i < Nq) ? rr[0] : -2;
        float qx = 0.f, qy = 0.f, qz = 0.f;
        if (n >= 0) {
            qx = sq[3 * li];
            qy = sq[3 * li + 1];
            qz = sq[3 * li + 2];
        }
        unsigned long long key = RF_NONE;
#pragma unroll 2
        for (int c = 0; c < n; ++c) {
            const int code = rr[2 + c];
            const int j0 = (code >> 4) * SC_CHUNK + SC_RUN * (code & 15) + 4 * tl;
#pragma unroll
            for (int e = 0; e < SC_RUN / RF_STEP; ++e) run4_key(key, qx, qy, qz, Pt, j0 + RF_STEP * e, Np);
        }
        int bj;
        float best;
        const bool found = team_result(key, bj, best);
        if (n >= 0 && tl == 0) {
            if (!found) {  // nothing comparable (non-finite data): first index
                bj = 0;
                best = canon_d2(qx, qy, qz, Pt);
            }
            idx[(size_t)t * Nq + i] = bj;
            dist[(size_t)t * Nq + i] = best;
        }
        if (tl == 0 && i < Nq) {
            my_cand += n >= 0 ? (unsigned)n : 0u;
            my_heavy += n < 0 ? 1u : 0u;
        }
    }
    flush_stats(cnt, stats, min(RF_QUERIES, Nq - blk.x * RF_QUERIES), my_cand,
                my_heavy, tl);
}

__global__ __launch_bounds__(RF_THREADS) void k_refine(RefineParams p) {
    refine_body(p, grid_blk_xcd());
}

// Column refine (b -> a): each candidate workgroup contributes its winning row group (8 rows per
// query tile: runs of 4, two per tile) or, when flagged ambiguous, all of its rows.
__device__ __forceinline__ void colrefine_body(const RefineParams &pr, const Blk &blk) {
    const float *__restrict__ B = pr.Q;
    const float *__restrict__ A = pr.P;
    const int Nb = pr.Nq, Na = pr.Np;
    const int32_t *__restrict__ crec = pr.rec;
    int32_t *__restrict__ idx = pr.idx;
    float *__restrict__ dist = pr.dist;
    unsigned long long *__restrict__ stats = pr.stats;
    __shared__ unsigned cnt[2];
    __shared__ int32_t srec[RF_QUERIES * CREC_INTS];
    __shared__ float sq[RF_QUERIES * 3];
    const int t = blk.y;
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __shared__ int bins[RF_BINS];
    __shared__ int16_t order[RF_QUERIES];
    stage_queries<CREC_INTS>(crec, B, t, Nb, blk.x * RF_QUERIES, srec, sq);
    __syncthreads();
    order_queries<CREC_INTS>(srec, min(RF_QUERIES, Nb - blk.x * RF_QUERIES), bins, order);
    const int team = threadIdx.x / RF_TEAM, tl = threadIdx.x % RF_TEAM;
    const float *At = A + (size_t)t * Na * 3;
    unsigned my_cand = 0, my_heavy = 0;
    for (int qq = 0; qq < RF_QUERIES / RF_TEAMS; ++qq) {
        const int lj = order[qq * RF_TEAMS + team];
        const int j = blk.x * RF_QUERIES + lj;
        const int32_t *rr = srec + lj * CREC_INTS;
        const int n = (j < Nb) ? rr[0] : -2;
        float qx = 0.f, qy = 0.f, qz = 0.f;
        if (n >= 0) {
            qx = sq[3 * lj];
            qy = sq[3 * lj + 1];
            qz = sq[3 * lj + 2];
        }
        unsigned long long key = RF_NONE;
#pragma unroll 2
        for (int e = 0; e < n; ++e) {
            const int code = rr[1 + e];
            const int wg = code >> 8, grp = code & 0x7f;
            const int wv = grp >> 1, h = grp & 1;
            if (code & 0x80) {  // ambiguous: every row of the workgroup, as runs of 4 rows
                for (int u = tl; u < sc_rows<true>() / 4; u += RF_TEAM)
                    run4_key(key, qx, qy, qz, At, wg * sc_rows<true>() + 4 * u, Na);
            } else if (tl < 2 * sc_atiles<true>()) {
                // the row group: runs of rows 16a + 4g + (0..3) of its wave, g in {h, h + 2}
                run4_key(key, qx, qy, qz, At,
                         wg * sc_rows<true>() + wv * (sc_atiles<true>() * 16) + 16 * (tl >> 1) +
                             4 * (h + 2 * (tl & 1)),
                         Na);
            }
        }
        int bi;
        float best;
        const bool found = team_result(key, bi, best);
        if (n >= 0 && tl == 0) {
            if (!found) {
                bi = 0;
                best = canon_d2(qx, qy, qz, At);
            }
            idx[(size_t)t * Nb + j] = bi;
            dist[(size_t)t * Nb + j] = best;
        }
        if (tl == 0 && j < Nb) {
            my_cand += n >= 0 ? (unsigned)n : 0u;
            my_heavy += n < 0 ? 1u : 0u;
        }
    }
    flush_stats(cnt, stats, min(RF_QUERIES, Nb - blk.x * RF_QUERIES), my_cand,
                my_heavy, tl);
}

__global__ __launch_bounds__(RF_THREADS) void k_colrefine(RefineParams p) {
    colrefine_body(p, grid_blk_xcd());
}

}  // namespace

static int padded_targets(int Np) { return ((Np + SC_CHUNK - 1) / SC_CHUNK) * SC_CHUNK; }

size_t screen_scratch_bytes(int T, int Na, int Nb) {
    // column partials exist only for the two-direction screen, whose row blocks they follow
    const size_t nwg = (size_t)(Na + sc_rows<true>() - 1) / sc_rows<true>();
    const size_t Nb_pad = padded_targets(Nb);
    return Arena::need((size_t)T, 4) * 4 +                           // norms, heavy counts
           Arena::need((size_t)T * Na, 4) + Arena::need((size_t)T * Nb, 4) +  // heavy lists
           Arena::need((size_t)T * Na * REC_INTS, 4) +                // row records
           Arena::need((size_t)T * Nb * CREC_INTS, 4) +               // column records
           Arena::need((size_t)T * Nb_pad * 3, sizeof(bf16x8)) +      // packed b operands
           Arena::need((size_t)T * Nb_pad, 4) +                       // their threshold slack
           Arena::need((size_t)T * nwg * Nb_pad, 2) +                 // column partial words
           std::max(nn_exact_list_scratch_bytes(T, Na, Nb), nn_exact_list_scratch_bytes(T, Nb, Na));
}

void launch_chamfer_screened(const float *a, int Na, const float *b, int Nb, int T,
                             int32_t *idx_a, float *dist_a, int32_t *idx_b, float *dist_b,
                             char *scratch, unsigned long long *stats, dc_ctx *prof,
                             hipStream_t s) {
    Arena ar;
    ar.base = scratch;
    ar.cap = screen_scratch_bytes(T, Na, Nb);
    const int nwg = (Na + sc_rows<true>() - 1) / sc_rows<true>();        // two directions
    const int nwg_rows = (Na + sc_rows<false>() - 1) / sc_rows<false>();  // one direction
    const int Nb_pad = padded_targets(Nb);
    float *nbmax = ar.take<float>((size_t)T);
    float *namax = ar.take<float>((size_t)T);
    int32_t *hcnt_a = ar.take<int32_t>((size_t)T);
    int32_t *hcnt_b = ar.take<int32_t>((size_t)T);
    int32_t *hlist_a = ar.take<int32_t>((size_t)T * Na);
    int32_t *hlist_b = ar.take<int32_t>((size_t)T * Nb);
    int32_t *rec = ar.take<int32_t>((size_t)T * Na * REC_INTS);
    int32_t *crec = ar.take<int32_t>((size_t)T * Nb * CREC_INTS);
    bf16x8 *packed = ar.take<bf16x8>((size_t)T * Nb_pad * 3);
    float *slack = ar.take<float>((size_t)T * Nb_pad);
    uint16_t *cpart = ar.take<uint16_t>((size_t)T * nwg * Nb_pad);
    char *exact_scratch = ar.take<char>(
        std::max(nn_exact_list_scratch_bytes(T, Na, Nb), nn_exact_list_scratch_bytes(T, Nb, Na)));
    NormMaxParams nm;
    nm.P = b;
    nm.Np = Nb;
    nm.out = nbmax;
    nm.heavy_cnt = hcnt_a;
    dispatch(KT_NORM_MAX, k_norm_max, dim3(T), NM_THREADS, nm, s);
    nm.P = a;
    nm.Np = Na;
    nm.out = namax;
    nm.heavy_cnt = hcnt_b;
    dispatch(KT_NORM_MAX, k_norm_max, dim3(T), NM_THREADS, nm, s);
    PackParams pk;
    pk.P = b;
    pk.nqmax = namax;
    pk.packed = packed;
    pk.slack = slack;
    pk.Np = Nb;
    pk.Np_pad = Nb_pad;
    dispatch(KT_PACK, k_pack_targets, dim3(Nb_pad / 256, T), 256, pk, s);
    // without b outputs (the unidirectional loss) only the row direction is screened
    const bool cols = idx_b != nullptr;
    {
        ProfScope ps(prof, 0, s);
        ScreenParams sp;
        sp.Q = a;
        sp.packed = packed;
        sp.slack = slack;
        sp.npmax = nbmax;
        sp.nqmax = namax;
        sp.rec = rec;
        sp.heavy_cnt = hcnt_a;
        sp.heavy_list = hlist_a;
        sp.cpart = cpart;
        sp.Nq = Na;
        sp.Np = Nb;
        sp.Np_pad = Nb_pad;
        if (cols)
            dispatch(KT_SCREEN, k_screen<true>, dim3(nwg, T), SC_THREADS, sp, s);
        else
            dispatch(KT_SCREEN_ROWS, k_screen<false>, dim3(nwg_rows, T), SC_THREADS, sp, s);
    }
    {
        ProfScope ps(prof, 1, s);
        RefineParams rp;
        rp.Q = a;
        rp.P = b;
        rp.rec = rec;
        rp.idx = idx_a;
        rp.dist = dist_a;
        rp.stats = stats;
        rp.Nq = Na;
        rp.Np = Nb;
        dispatch(KT_REFINE, k_refine, dim3((Na + RF_QUERIES - 1) / RF_QUERIES, T), RF_THREADS, rp,
                 s);
        launch_nn_exact_list(a, Na, b, Nb, T, hlist_a, hcnt_a, idx_a, dist_a, exact_scratch, s);
        if (!cols) return;
        ColmergeParams cm;
        cm.P = b;
        cm.slack = slack;
        cm.cpart = cpart;
        cm.nqmax = namax;
        cm.npmax = nbmax;
        cm.crec = crec;
        cm.heavy_cnt = hcnt_b;
        cm.heavy_list = hlist_b;
        cm.Np = Nb;
        cm.Np_pad = Nb_pad;
        cm.nwg = nwg;
        dispatch(KT_COLMERGE, k_colmerge,
                 dim3((Nb + CM_THREADS * CM_TPT - 1) / (CM_THREADS * CM_TPT), T), CM_THREADS, cm, s);
        RefineParams cr;
        cr.Q = b;
        cr.P = a;
        cr.rec = crec;
        cr.idx = idx_b;
        cr.dist = dist_b;
        cr.stats = stats;
        cr.Nq = Nb;
        cr.Np = Na;
        dispatch(KT_COLREFINE, k_colrefine, dim3((Nb + RF_QUERIES - 1) / RF_QUERIES, T),
                 RF_THREADS, cr, s);
        launch_nn_exact_list(b, Nb, a, Na, T, hlist_b, hcnt_b, idx_b, dist_b, exact_scratch, s);
    }
}

void register_screen_kernels(BatchedKernel *table) {
    table[KT_NORM_MAX] = batched_kernel<NormMaxParams, norm_max_body, NM_THREADS, 256>();
    table[KT_PACK] = batched_kernel<PackParams, pack_body, 256, 1024>();
    // two screen workgroups per compute unit fit the batched kernel's registers (forcing three
    // spills registers and measured slower)
    // persistent blocks = the workgroups that fit at once (two or three per compute unit), with
    // the same register bounds as the direct kernels so that they all stay resident
    table[KT_SCREEN] = batched_kernel<ScreenParams, screen_body<true>, SC_THREADS, 512,
                                      sc_atiles<true>() <= 4 ? 3 : 2>();
    table[KT_SCREEN_ROWS] = batched_kernel<ScreenParams, screen_body<false>, SC_THREADS,
                                           sc_atiles<false>() <= 4 ? 768 : 512,
                                           sc_atiles<false>() <= 4 ? 3 : 2>();
    // six waves per SIMD (at most 80 registers, which the refine bodies need without spilling):
    // 1,536 blocks
    table[KT_REFINE] = batched_kernel<RefineParams, refine_body, RF_THREADS, 1536, 6>();
    table[KT_COLMERGE] = batched_kernel<ColmergeParams, colmerge_body, CM_THREADS, 1024>();
    table[KT_COLREFINE] = batched_kernel<RefineParams, colrefine_body, RF_THREADS, 1536, 6>();
}

}  // namespace dc
