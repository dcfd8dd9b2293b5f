// bf16 matrix-core screen + certified exact refine for the all-pairs nearest neighbour
// (Sec. III-A, Eq. 1/2): the same indices as the exact single-precision search, found faster.
//
// Screen (k_screen): the squared distance is expanded as s_ij = |q_i|^2 + |p_j|^2 - 2 q_i.p_j and
// evaluated as one K=32 dot product per pair on v_mfma_f32_16x16x32_bf16 with fp32 accumulation.
// Each float coordinate is split exactly into three bf16 parts (x = h + m + l), and the six
// products hH, hM, mH, hL, lH, mM per coordinate (18 K-slots) plus the two norms, each split in
// three (6 K-slots), fill 24 of the 32 K-slots; the matrix unit does the whole distance, the vector
// unit only keeps minimums (one v_min3 per two pairs).  Query rows stay in registers (64 per wave,
// four 16-row tiles); targets stream through LDS in groups of 256, their bf16 operand built while
// staging.  Targets are laid out so that, inside each chunk of 1024, result column c of the 64
// tiles holds the 64 consecutive targets [64c, 64c+64): a (column, chunk) "slot group" is one
// contiguous run.  For every (lane, row) the kernel keeps the minimum of each of its slot groups,
// and the two best groups and the third-best value.
// Certificate: with a rigorous bound e_ij <= C (|q_i|^2 + |p_j|^2) on |s_ij - d_ij| (bf16 splits
// exact, products exact, at most 24 roundings of the fp32 accumulator at 2^-23), every index whose
// canonical float distance can equal the minimum has s_ij <= m_i + Delta_i, where m_i is the
// row's screened minimum and Delta_i bounds the error at the screened winner and at the canonical
// winner (both lie within sqrt(m_i + e) of q_i, which bounds their norms).  Slot groups whose
// minimum passes that test are candidates.  A row is "heavy" (searched exhaustively by the exact
// kernel) if a slot has three passing groups, if it has more than MAXC candidates, or if its
// minimum is not finite; heavy rows are appended to a per-frame list.
// Refine (k_refine): one lane per light query evaluates the canonical distance
// fma(dz,dz,fma(dy,dy,dx*dx)) over its candidate groups and keeps the lexicographic
// (distance, index) minimum, which is exactly the argmin of the exhaustive search with the
// smallest-index rule.
#include "dc_internal.h"

namespace dc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int SC_WAVES = 4;
constexpr int SC_THREADS = 64 * SC_WAVES;
constexpr int SC_ATILES = 4;                            // 16-row tiles per wave
constexpr int SC_ROWS = SC_WAVES * SC_ATILES * 16;       // 256 query rows per workgroup
constexpr int SC_STAGE = 256;                            // targets staged in LDS per step
constexpr int SC_CHUNK = 1024;                           // targets per tracking chunk
constexpr int SC_ROWPAD = 17;                            // LDS entries per staged tile
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
__global__ __launch_bounds__(256) void k_pack_targets(const float *__restrict__ P, int Np,
                                                      int Np_pad, bf16x8 *__restrict__ packed) {
    const int t = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= Np_pad) return;
    const bool valid = j < Np;
    const float *p = P + ((size_t)t * Np + (valid ? j : 0)) * 3;
    __bf16 v[32];
    target_vector(valid ? p[0] : 0.f, valid ? p[1] : 0.f, valid ? p[2] : 0.f, valid, v);
    bf16x8 *o = packed + ((size_t)t * Np_pad + j) * 3;
    o[0] = pick8(v, 0);
    o[1] = pick8(v, 1);
    o[2] = pick8(v, 2);
}

// largest squared norm of each frame's targets (for the certificate)
__global__ __launch_bounds__(256) void k_norm_max(const float *__restrict__ P, int Np,
                                                  float *__restrict__ out,
                                                  int32_t *__restrict__ heavy_cnt) {
    __shared__ float red[256];
    const int t = blockIdx.x;
    if (threadIdx.x == 0) heavy_cnt[t] = 0;
    const float *pt = P + (size_t)t * Np * 3;
    float m = 0.f;
    for (int j = threadIdx.x; j < Np; j += 256)
        m = fmaxf(m, norm2(pt[3 * (size_t)j], pt[3 * (size_t)j + 1], pt[3 * (size_t)j + 2]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[t] = red[0];
}

__global__ __launch_bounds__(SC_THREADS) void k_screen(const float *__restrict__ Q, int Nq,
                                                       const bf16x8 *__restrict__ packed,
                                                       int Np, int Np_pad,
                                                       const float *__restrict__ npmax,
                                                       int32_t *__restrict__ rec,
                                                       int32_t *__restrict__ heavy_cnt,
                                                       int32_t *__restrict__ heavy_list) {
    // [buffer][K-chunk][entry] -> 16 bytes.  Entry 17*bt + c holds tile bt, result column c: the
    // operand reads (16 columns of one tile) are consecutive and the staging stores (8 tiles of
    // one column, 272 bytes apart) fall in distinct banks; the read address is a per-lane base
    // plus a compile-time offset.  K-chunk 3 is all zeros on the query side and is not stored.
    __shared__ bf16x8 stage[2][3][SC_ROWPAD * 16];
    const int t = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;   // K-chunk of the operands; row group of the result
    const int col = lane & 15; // row of the A operand; column (slot) of the result
    const float *Qt = Q + (size_t)t * Nq * 3;
    const bf16x8 *Bt = packed + (size_t)t * Np_pad * 3;
    const int row0 = blockIdx.x * SC_ROWS + wave * (SC_ATILES * 16);

    // query operands, held for the whole sweep
    bf16x8 A[SC_ATILES];
#pragma unroll
    for (int a = 0; a < SC_ATILES; ++a) {
        const int r = row0 + 16 * a + col;
        __bf16 v[32];
        if (r < Nq)
            query_vector(Qt[3 * (size_t)r], Qt[3 * (size_t)r + 1], Qt[3 * (size_t)r + 2], v);
        else
            query_vector(0.f, 0.f, 0.f, v);
        A[a] = pick8(v, g);
    }

    const float inf = __builtin_inff();
    float m[SC_ATILES][4], b1[SC_ATILES][4], b2[SC_ATILES][4], b3[SC_ATILES][4];
    int c1[SC_ATILES][4], c2[SC_ATILES][4];
#pragma unroll
    for (int a = 0; a < SC_ATILES; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            m[a][r] = inf;
            b1[a][r] = inf;
            b2[a][r] = inf;
            b3[a][r] = inf;
            c1[a][r] = -1;
            c2[a][r] = -1;
        }
    const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
    const int nstage = Np_pad / SC_STAGE;
    // staging position of this thread: tile-local position (btl, c) of a stage holds target
    // 64c + 16*(stage in chunk) + btl of the chunk, so result column c of a chunk is the
    // contiguous run [64c, 64c+64)
    const int sc = threadIdx.x >> 4, sbtl = threadIdx.x & 15;
    const int spos = sbtl * SC_ROWPAD + sc;
    auto target_of = [&](int st) {
        return (st / (SC_CHUNK / SC_STAGE)) * SC_CHUNK + 64 * sc + 16 * (st % (SC_CHUNK / SC_STAGE)) +
               sbtl;
    };
    // register prefetch of the next stage's operands, double-buffered LDS: one barrier per stage
    bf16x8 q0, q1, q2;
    {
        const bf16x8 *src = Bt + (size_t)target_of(0) * 3;
        q0 = src[0];
        q1 = src[1];
        q2 = src[2];
    }
    const int gk = (g == 3) ? 0 : g;
    for (int st = 0; st < nstage; ++st) {
        const int buf = st & 1;
        stage[buf][0][spos] = q0;
        stage[buf][1][spos] = q1;
        stage[buf][2][spos] = q2;
        if (st + 1 < nstage) {
            const bf16x8 *src = Bt + (size_t)target_of(st + 1) * 3;
            q0 = src[0];
            q1 = src[1];
            q2 = src[2];
        }
        __syncthreads();
        // lanes of K-group 3 hold an all-zero query operand, so any finite staged operand gives
        // them zero products: they read K-chunk 0 instead of a stored zero chunk
        const bf16x8 *sb = &stage[buf][gk][col];
#pragma unroll 2
        for (int bt = 0; bt < SC_STAGE / 16; bt += 2) {
            const bf16x8 B0 = sb[bt * SC_ROWPAD];
            const bf16x8 B1 = sb[(bt + 1) * SC_ROWPAD];
#pragma unroll
            for (int a = 0; a < SC_ATILES; ++a) {
                const floatx4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a], B0, zero, 0, 0, 0);
                const floatx4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a], B1, zero, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) m[a][r] = fminf(fminf(m[a][r], d0[r]), d1[r]);
            }
        }
        if ((st + 1) % (SC_CHUNK / SC_STAGE) == 0) {  // end of a tracking chunk
            const int k = st / (SC_CHUNK / SC_STAGE);
#pragma unroll
            for (int a = 0; a < SC_ATILES; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float x = m[a][r];
                    const bool t1 = x < b1[a][r];
                    const bool t2 = x < b2[a][r];
                    b3[a][r] = __builtin_amdgcn_fmed3f(x, b2[a][r], b3[a][r]);
                    b2[a][r] = __builtin_amdgcn_fmed3f(x, b1[a][r], b2[a][r]);
                    b1[a][r] = fminf(x, b1[a][r]);
                    c2[a][r] = t1 ? c1[a][r] : (t2 ? k : c2[a][r]);
                    c1[a][r] = t1 ? k : c1[a][r];
                    m[a][r] = inf;
                }
        }
    }

    // certificate and candidate records; the 16 lanes of a group share one row per (a, r)
    const float npm = npmax[t];
    const unsigned long long gmask = 0xFFFFull << (16 * g);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int a = 0; a < SC_ATILES; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = row0 + 16 * a + 4 * g + r;
            float mi = b1[a][r];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) mi = fminf(mi, __shfl_xor(mi, off, 64));
            float nq = 0.f;
            if (row < Nq)
                nq = norm2(Qt[3 * (size_t)row], Qt[3 * (size_t)row + 1], Qt[3 * (size_t)row + 2]);
            // Delta: error bound at the screened winner (E1) and at the canonical winner (E2);
            // each winner lies within sqrt(distance) of q, which bounds its squared norm
            const float up = 1.0001f;
            const float qn = __builtin_sqrtf(nq) * up;
            const float mp = fmaxf(mi, 0.f);
            const float e0 = (SCREEN_C * (nq + npm) + SCREEN_TAU) * up;
            const float r0 = qn + __builtin_sqrtf(mp + e0) * up;
            const float e1 = (SCREEN_C * (nq + r0 * r0) + SCREEN_TAU) * up;
            const float d1 = (mp + e1) * (1.0f + CANON_U13) * up;
            const float r1 = qn + __builtin_sqrtf(d1) * up;
            const float e2 = (SCREEN_C * (nq + r1 * r1) + SCREEN_TAU) * up;
            const float theta = (mi + e1 + e2 + CANON_U13 * (mp + e1)) * up + SCREEN_TAU;
            const bool finite = __builtin_isfinite(mi) && __builtin_isfinite(theta) &&
                                __builtin_isfinite(npm);
            const bool k1 = finite && c1[a][r] >= 0 && b1[a][r] <= theta;
            const bool k2 = finite && c2[a][r] >= 0 && b2[a][r] <= theta;
            const bool over = finite && b3[a][r] <= theta;
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
                    if (k1) rr[2 + off] = (c1[a][r] << 4) | col;
                    if (k2) rr[2 + off + (k1 ? 1 : 0)] = (c2[a][r] << 4) | col;
                }
            }
        }
}

__device__ __forceinline__ float canon_d2(float qx, float qy, float qz, const float *p) {
    const float dx = qx - p[0];
    const float dy = qy - p[1];
    const float dz = qz - p[2];
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

constexpr int RF_THREADS = 256;
constexpr int RF_TEAM = 16;                         // lanes per query
constexpr int RF_TEAMS = RF_THREADS / RF_TEAM;
constexpr int RF_QUERIES = 256;                     // queries per workgroup (16 per team)

// Exact re-evaluation of the candidate groups of light rows (heavy rows are left to the exact
// kernel and skipped here).  A team of 16 lanes takes one query; in each 64-target group a lane
// evaluates 4 consecutive targets (48 contiguous bytes), then the team reduces the lexicographic
// (distance, index) minimum.
__global__ __launch_bounds__(RF_THREADS) void k_refine(const float *__restrict__ Q, int Nq,
                                                       const float *__restrict__ P, int Np,
                                                       const int32_t *__restrict__ rec,
                                                       int32_t *__restrict__ idx,
                                                       float *__restrict__ dist,
                                                       unsigned long long *__restrict__ stats) {
    __shared__ unsigned cnt[2];
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int t = blockIdx.y;
    const int team = threadIdx.x / RF_TEAM, tl = threadIdx.x % RF_TEAM;
    const float *Pt = P + (size_t)t * Np * 3;
    unsigned my_cand = 0, my_heavy = 0;
    for (int qq = 0; qq < RF_QUERIES / RF_TEAMS; ++qq) {
    const int i = blockIdx.x * RF_QUERIES + qq * RF_TEAMS + team;
    const int32_t *rr = rec + ((size_t)t * Nq + min(i, Nq - 1)) * REC_INTS;
    const int n = (i < Nq) ? rr[0] : -2;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (n >= 0) {
        const float *q = Q + ((size_t)t * Nq + i) * 3;
        qx = q[0];
        qy = q[1];
        qz = q[2];
    }
    float best = __builtin_inff();
    int bj = 0x7fffffff;
    for (int e = 0; e < n; ++e) {
        const int code = rr[2 + e];
        const int j = (code >> 4) * SC_CHUNK + 64 * (code & 15) + 4 * tl;
        float c[12];
        if (j + 3 < Np) {
            const float4 *p4 = reinterpret_cast<const float4 *>(Pt + 3 * (size_t)j);
            const float4 u0 = p4[0], u1 = p4[1], u2 = p4[2];
            c[0] = u0.x; c[1] = u0.y; c[2] = u0.z; c[3] = u0.w;
            c[4] = u1.x; c[5] = u1.y; c[6] = u1.z; c[7] = u1.w;
            c[8] = u2.x; c[9] = u2.y; c[10] = u2.z; c[11] = u2.w;
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) c[k] = (j + k / 3 < Np) ? Pt[3 * (size_t)j + k] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (j + k < Np) {
                const float d = canon_d2(qx, qy, qz, c + 3 * k);
                if (d < best || (d == best && j + k < bj)) {
                    best = d;
                    bj = j + k;
                }
            }
        }
    }
#pragma unroll
    for (int off = RF_TEAM / 2; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off, RF_TEAM);
        const int oj = __shfl_xor(bj, off, RF_TEAM);
        if (ob < best || (ob == best && oj < bj)) {
            best = ob;
            bj = oj;
        }
    }
    if (n >= 0 && tl == 0) {
        if (bj == 0x7fffffff) {  // nothing comparable (non-finite data): first index
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
    if (stats) {
        if (tl == 0) {
            atomicAdd(&cnt[0], my_cand);
            atomicAdd(&cnt[1], my_heavy);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int live = min(RF_QUERIES, Nq - (int)blockIdx.x * RF_QUERIES);
            atomicAdd(&stats[0], (unsigned long long)live);
            atomicAdd(&stats[1], (unsigned long long)cnt[0]);
            atomicAdd(&stats[2], (unsigned long long)cnt[1]);
        }
    }
}

}  // namespace

bool screen_available() { return true; }

static int padded_targets(int Np) { return ((Np + SC_CHUNK - 1) / SC_CHUNK) * SC_CHUNK; }

size_t screen_scratch_bytes(int T, int Nq, int Np) {
    return Arena::need((size_t)T, 4) * 2 + Arena::need((size_t)T * Nq, 4) +
           Arena::need((size_t)T * Nq * REC_INTS, 4) + nn_exact_list_scratch_bytes(T, Nq, Np) +
           Arena::need((size_t)T * padded_targets(Np) * 3, sizeof(bf16x8));
}

void launch_nn_screened(const float *Q, int Nq, const float *P, int Np, int T, int32_t *idx,
                        float *dist, char *scratch, unsigned long long *stats, dc_ctx *prof,
                        hipStream_t s) {
    Arena ar;
    ar.base = scratch;
    ar.cap = screen_scratch_bytes(T, Nq, Np);
    float *npmax = ar.take<float>((size_t)T);
    int32_t *heavy_cnt = ar.take<int32_t>((size_t)T);
    int32_t *heavy_list = ar.take<int32_t>((size_t)T * Nq);
    int32_t *rec = ar.take<int32_t>((size_t)T * Nq * REC_INTS);
    char *exact_scratch = ar.take<char>(nn_exact_list_scratch_bytes(T, Nq, Np));
    const int Np_pad = padded_targets(Np);
    bf16x8 *packed = ar.take<bf16x8>((size_t)T * Np_pad * 3);
    hipLaunchKernelGGL(k_norm_max, dim3(T), dim3(256), 0, s, P, Np, npmax, heavy_cnt);
    hipLaunchKernelGGL(k_pack_targets, dim3(Np_pad / 256, T), dim3(256), 0, s, P, Np, Np_pad,
                       packed);
    {
        ProfScope ps(prof, 0, s);
        hipLaunchKernelGGL(k_screen, dim3((Nq + SC_ROWS - 1) / SC_ROWS, T), dim3(SC_THREADS), 0,
                           s, Q, Nq, packed, Np, Np_pad, npmax, rec, heavy_cnt, heavy_list);
    }
    {
        ProfScope ps(prof, 1, s);
        hipLaunchKernelGGL(k_refine, dim3((Nq + RF_QUERIES - 1) / RF_QUERIES, T),
                           dim3(RF_THREADS), 0, s, Q, Nq, P, Np, rec, idx, dist, stats);
        launch_nn_exact_list(Q, Nq, P, Np, T, heavy_list, heavy_cnt, idx, dist, exact_scratch, s);
    }
}

}  // namespace dc
