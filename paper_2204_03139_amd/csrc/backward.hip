// Backward passes: the Chamfer gradient through the saved neighbours (Sec. III-A, Eq. 1/2) and
// the sampling gradient through Eq. 4 (Sec. III-B).  Both are gathers over segments built by the
// stable atomic-free sort, summed in increasing index order and in double (each output rounded
// once to float), so every result is bitwise reproducible, independent of scheduling, and within a
// few units of 2^-24 of the sum of its terms' magnitudes however long a segment is.
#include "batch.h"

namespace dc {
namespace {

constexpr int BW_THREADS = 256;

// g_x[t,i] = g_t w_t ( cs * (x_i - y_{nn_x[i]}) + cm * sum_{j: nn_y[j]=i} (x_i - y_j) )
// for x = a (cs = 2 alpha, cm = 2 beta) or x = b (cs = 2 beta, cm = 2 alpha).
struct ChamferBwdParams {
    const double *grad_loss;
    const float *X;
    const float *Y;
    const int32_t *nn_x;
    const int32_t *ystart;        // [T][Nx + 1]: first sorted position of each neighbour in x
    const int32_t *yvals_sorted;
    const float *frame_w;
    float *gX;
    double cself, cmutual;
    int Nx, Ny;
};

__device__ __forceinline__ void chamfer_bwd_body(const ChamferBwdParams &pr, const Blk &blk) {
    const double *__restrict__ grad_loss = pr.grad_loss;
    const float *__restrict__ X = pr.X;
    const float *__restrict__ Y = pr.Y;
    const int32_t *__restrict__ nn_x = pr.nn_x;
    const int32_t *__restrict__ ystart = pr.ystart;
    const int32_t *__restrict__ yvals_sorted = pr.yvals_sorted;
    const int Nx = pr.Nx, Ny = pr.Ny;
    const double cself = pr.cself, cmutual = pr.cmutual;
    const float *__restrict__ frame_w = pr.frame_w;
    float *__restrict__ gX = pr.gX;
    const int t = blk.y;
    const int i = blk.x * BW_THREADS + threadIdx.x;
    if (i >= Nx) return;
    const double g = grad_loss[t] * (frame_w ? (double)frame_w[t] : 1.0);
    const double cs = cself * g;
    const double cm = cmutual * g;
    const float *xt = X + (size_t)t * Nx * 3;
    const float *yt = Y + (size_t)t * Ny * 3;
    // in double (each difference of two floats is exact there) and rounded once to float: the
    // result stays within a few units of 2^-24 of the sum of the terms' magnitudes however many
    // points share this neighbour
    const double x0 = xt[3 * (size_t)i], x1 = xt[3 * (size_t)i + 1], x2 = xt[3 * (size_t)i + 2];
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    // the own-neighbour term exists only when cs != 0 (nn_x may be NULL otherwise: the b side of
    // the unidirectional loss has no neighbour indices)
    const int jn = (cs != 0.0) ? nn_x[(size_t)t * Nx + i] : -1;
    if ((unsigned)jn < (unsigned)Ny) {  // indices outside [0, Ny) contribute nothing
        const int j = jn;
        g0 = cs * (x0 - (double)yt[3 * (size_t)j]);
        g1 = cs * (x1 - (double)yt[3 * (size_t)j + 1]);
        g2 = cs * (x2 - (double)yt[3 * (size_t)j + 2]);
    }
    if (cm != 0.0) {
        const int32_t *vs = yvals_sorted + (size_t)t * Ny;
        const int32_t *st = ystart + (size_t)t * (Nx + 1);
        const int lo = st[i], hi = st[i + 1];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int p = lo; p < hi; ++p) {
            const int j = vs[p];
            if (j < 0) continue;  // a neighbour index outside [0, Nx): contributes nothing
            s0 += x0 - (double)yt[3 * (size_t)j];
            s1 += x1 - (double)yt[3 * (size_t)j + 1];
            s2 += x2 - (double)yt[3 * (size_t)j + 2];
        }
        g0 += cm * s0;
        g1 += cm * s1;
        g2 += cm * s2;
    }
    float *o = gX + ((size_t)t * Nx + i) * 3;
    o[0] = (float)g0;
    o[1] = (float)g1;
    o[2] = (float)g2;
}

__global__ __launch_bounds__(BW_THREADS) void k_chamfer_bwd(ChamferBwdParams p) {
    chamfer_bwd_body(p, grid_blk_xcd());
}

// start[t][k] = first position of the sorted keys of frame t whose key is >= k, for k in [0, K]
// (the sort clamps its keys into [0, K]).  The thread of position q in [0, N] writes the entries
// of the keys in (key[q-1], key[q]] (key[-1] = -1, key[N] = K), so every entry is written exactly
// once, by adjacent differences instead of a binary search per key.
struct BoundsParams {
    const int32_t *sorted;
    int32_t *start;
    int N, K;
};

__device__ __forceinline__ void bounds_body(const BoundsParams &p, const Blk &blk) {
    const int t = blk.y;
    const int q = blk.x * BW_THREADS + threadIdx.x;
    if (q > p.N) return;
    const int32_t *s = p.sorted + (size_t)t * p.N;
    const int lo = q == 0 ? -1 : min(s[q - 1], p.K);
    const int hi = q == p.N ? p.K : min(s[q], p.K);
    int32_t *st = p.start + (size_t)t * (p.K + 1);
    for (int k = lo + 1; k <= hi; ++k) st[k] = q;
}

__global__ __launch_bounds__(BW_THREADS) void k_bounds(BoundsParams p) { bounds_body(p, grid_blk()); }

// per face and corner: fg[t,f,c] = sum over the points i of face f, in increasing i, of
// bary[t,i,c] * g[t,i]
struct FaceGradParams {
    const float *gpts;
    const float *bary;
    const int32_t *pts_by_face;
    const int32_t *face_start;
    float *fg;
    int F, N;
};

__device__ __forceinline__ void face_grad_body(const FaceGradParams &pr, const Blk &blk) {
    const float *__restrict__ gpts = pr.gpts;
    const float *__restrict__ bary = pr.bary;
    const int32_t *__restrict__ pts_by_face = pr.pts_by_face;
    const int32_t *__restrict__ face_start = pr.face_start;
    const int F = pr.F, N = pr.N;
    float *__restrict__ fg = pr.fg;
    const int t = blk.y;
    const int f = blk.x * BW_THREADS + threadIdx.x;
    if (f >= F) return;
    const int32_t *fs = face_start + (size_t)t * (F + 1);
    const int32_t *pf = pts_by_face + (size_t)t * N;
    const float *gt = gpts + (size_t)t * N * 3;
    const float *bt = bary + (size_t)t * N * 3;
    // in double (a product of two floats is exact there), rounded once to float per (face, corner)
    double acc[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int p = fs[f]; p < fs[f + 1]; ++p) {
        const int i = pf[p];
        const double g0 = gt[3 * (size_t)i], g1 = gt[3 * (size_t)i + 1], g2 = gt[3 * (size_t)i + 2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double w = bt[3 * (size_t)i + c];
            acc[c][0] = __builtin_fma(w, g0, acc[c][0]);
            acc[c][1] = __builtin_fma(w, g1, acc[c][1]);
            acc[c][2] = __builtin_fma(w, g2, acc[c][2]);
        }
    }
    float *o = fg + ((size_t)t * F + f) * 9;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) o[3 * c + d] = (float)acc[c][d];
}

__global__ __launch_bounds__(BW_THREADS) void k_face_grad(FaceGradParams p) {
    face_grad_body(p, grid_blk_xcd());
}

// grad_verts[t,v] = sum over the incident (face f, corner c), in increasing (f, c), of fg[t,f,c]
struct VertexGradParams {
    const float *fg;
    const int32_t *corners_by_vertex;
    const int32_t *vert_start;
    float *gverts;
    int V, F;
};

__device__ __forceinline__ void vertex_grad_body(const VertexGradParams &pr, const Blk &blk) {
    const float *__restrict__ fg = pr.fg;
    const int32_t *__restrict__ corners_by_vertex = pr.corners_by_vertex;
    const int32_t *__restrict__ vert_start = pr.vert_start;
    const int V = pr.V, F = pr.F;
    float *__restrict__ gverts = pr.gverts;
    const int t = blk.y;
    const int v = blk.x * BW_THREADS + threadIdx.x;
    if (v >= V) return;
    const float *ft = fg + (size_t)t * F * 9;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;  // in double, rounded once to float
    for (int q = vert_start[v]; q < vert_start[v + 1]; ++q) {
        const int fc = corners_by_vertex[q];  // 3 f + c
        a0 += ft[3 * (size_t)fc];
        a1 += ft[3 * (size_t)fc + 1];
        a2 += ft[3 * (size_t)fc + 2];
    }
    float *o = gverts + ((size_t)t * V + v) * 3;
    o[0] = (float)a0;
    o[1] = (float)a1;
    o[2] = (float)a2;
}

__global__ __launch_bounds__(BW_THREADS) void k_vertex_grad(VertexGradParams p) {
    vertex_grad_body(p, grid_blk_xcd());
}

}  // namespace

size_t chamfer_bwd_scratch_bytes(int T, int Na, int Nb, bool want_b) {
    size_t s = 2 * Arena::need((size_t)T * Nb, 4) + segsort_scratch_bytes(T, Nb) +
               Arena::need((size_t)T * (Na + 1), 4);
    if (want_b)
        s += 2 * Arena::need((size_t)T * Na, 4) + segsort_scratch_bytes(T, Na) +
             Arena::need((size_t)T * (Nb + 1), 4);
    return s;
}

void launch_chamfer_bwd(const double *grad_loss, const float *a, const float *b,
                        const int32_t *idx_a, const int32_t *idx_b, int T, int Na, int Nb,
                        int reduction, const float *frame_w, float *grad_a, float *grad_b,
                        char *scratch, hipStream_t s) {
    const bool eq2 = reduction == DC_RED_SIM2REAL_SUM;
    const double alpha = eq2 ? 1.0 : 1.0 / (double)Na;
    const double beta = eq2 ? 0.0 : 1.0 / (double)Nb;
    Arena ar;
    ar.base = scratch;
    ar.cap = chamfer_bwd_scratch_bytes(T, Na, Nb, grad_b != nullptr);
    // segments of b grouped by their neighbour in a (needed when beta != 0)
    int32_t *kb = ar.take<int32_t>((size_t)T * Nb);
    int32_t *vb = ar.take<int32_t>((size_t)T * Nb);
    char *ssb = ar.take<char>(segsort_scratch_bytes(T, Nb));
    int32_t *sb = ar.take<int32_t>((size_t)T * (Na + 1));
    if (beta != 0.0) {
        // valid neighbours lie in [0, Na): Na - 1 is the key limit, out-of-range ones are marked
        launch_segsort(idx_b, T, Nb, Na - 1, kb, vb, ssb, s, true);
        BoundsParams bp;
        bp.sorted = kb;
        bp.start = sb;
        bp.N = Nb;
        bp.K = Na;
        dispatch(KT_BOUNDS, k_bounds, dim3((Nb + BW_THREADS) / BW_THREADS, T), BW_THREADS, bp, s);
    }
    ChamferBwdParams cp;
    cp.grad_loss = grad_loss;
    cp.X = a;
    cp.Y = b;
    cp.nn_x = idx_a;
    cp.ystart = sb;
    cp.yvals_sorted = vb;
    cp.frame_w = frame_w;
    cp.gX = grad_a;
    cp.cself = 2.0 * alpha;
    cp.cmutual = 2.0 * beta;
    cp.Nx = Na;
    cp.Ny = Nb;
    dispatch(KT_CHAMFER_BWD, k_chamfer_bwd, dim3((Na + BW_THREADS - 1) / BW_THREADS, T),
             BW_THREADS, cp, s);
    if (grad_b) {
        int32_t *ka = ar.take<int32_t>((size_t)T * Na);
        int32_t *va = ar.take<int32_t>((size_t)T * Na);
        char *ssa = ar.take<char>(segsort_scratch_bytes(T, Na));
        int32_t *sa = ar.take<int32_t>((size_t)T * (Nb + 1));
        launch_segsort(idx_a, T, Na, Nb - 1, ka, va, ssa, s, true);
        BoundsParams bq;
        bq.sorted = ka;
        bq.start = sa;
        bq.N = Na;
        bq.K = Nb;
        dispatch(KT_BOUNDS, k_bounds, dim3((Na + BW_THREADS) / BW_THREADS, T), BW_THREADS, bq, s);
        ChamferBwdParams cq;
        cq.grad_loss = grad_loss;
        cq.X = b;
        cq.Y = a;
        cq.nn_x = idx_b;
        cq.ystart = sa;
        cq.yvals_sorted = va;
        cq.frame_w = frame_w;
        cq.gX = grad_b;
        cq.cself = 2.0 * beta;
        cq.cmutual = 2.0 * alpha;
        cq.Nx = Nb;
        cq.Ny = Na;
        dispatch(KT_CHAMFER_BWD, k_chamfer_bwd, dim3((Nb + BW_THREADS - 1) / BW_THREADS, T),
                 BW_THREADS, cq, s);
    }
}

size_t sample_bwd_scratch_bytes(int T, int V, int F, int N) {
    return 2 * Arena::need((size_t)T * N, 4) + segsort_scratch_bytes(T, N) +
           Arena::need((size_t)T * (F + 1), 4) + 2 * Arena::need((size_t)3 * F, 4) +
           segsort_scratch_bytes(1, 3 * F) + Arena::need((size_t)V + 1, 4) +
           Arena::need((size_t)T * F * 9, 4);
}

void launch_sample_bwd(const float *grad_points, const int32_t *faces, const int32_t *face_idx,
                       const float *bary, int T, int V, int F, int N, float *grad_verts,
                       char *scratch, hipStream_t s) {
    Arena ar;
    ar.base = scratch;
    ar.cap = sample_bwd_scratch_bytes(T, V, F, N);
    int32_t *fk = ar.take<int32_t>((size_t)T * N);
    int32_t *fv = ar.take<int32_t>((size_t)T * N);
    char *ss1 = ar.take<char>(segsort_scratch_bytes(T, N));
    int32_t *fstart = ar.take<int32_t>((size_t)T * (F + 1));
    int32_t *ck = ar.take<int32_t>((size_t)3 * F);
    int32_t *cv = ar.take<int32_t>((size_t)3 * F);
    char *ss2 = ar.take<char>(segsort_scratch_bytes(1, 3 * F));
    int32_t *vstart = ar.take<int32_t>((size_t)V + 1);
    float *fg = ar.take<float>((size_t)T * F * 9);
    // points grouped by face (face -1 of a degenerate frame sorts last, as key F, and is unused)
    launch_segsort(face_idx, T, N, F, fk, fv, ss1, s);
    BoundsParams bp;
    bp.sorted = fk;
    bp.start = fstart;
    bp.N = N;
    bp.K = F;
    dispatch(KT_BOUNDS, k_bounds, dim3((N + BW_THREADS) / BW_THREADS, T), BW_THREADS, bp, s);
    // (face, corner) slots grouped by vertex: the vertex-incidence CSR of the topology
    launch_segsort(faces, 1, 3 * F, V, ck, cv, ss2, s);
    bp.sorted = ck;
    bp.start = vstart;
    bp.N = 3 * F;
    bp.K = V;
    dispatch(KT_BOUNDS, k_bounds, dim3((3 * F + BW_THREADS) / BW_THREADS, 1), BW_THREADS, bp, s);
    FaceGradParams fp;
    fp.gpts = grad_points;
    fp.bary = bary;
    fp.pts_by_face = fv;
    fp.face_start = fstart;
    fp.fg = fg;
    fp.F = F;
    fp.N = N;
    dispatch(KT_FACE_GRAD, k_face_grad, dim3((F + BW_THREADS - 1) / BW_THREADS, T), BW_THREADS, fp,
             s);
    VertexGradParams vp;
    vp.fg = fg;
    vp.corners_by_vertex = cv;
    vp.vert_start = vstart;
    vp.gverts = grad_verts;
    vp.V = V;
    vp.F = F;
    dispatch(KT_VERTEX_GRAD, k_vertex_grad, dim3((V + BW_THREADS - 1) / BW_THREADS, T), BW_THREADS,
             vp, s);
}

void register_backward_kernels(BatchedKernel *table) {
    table[KT_CHAMFER_BWD] = batched_kernel<ChamferBwdParams, chamfer_bwd_body, BW_THREADS, 1024>();
    table[KT_BOUNDS] = batched_kernel<BoundsParams, bounds_body, BW_THREADS, 512>();
    table[KT_FACE_GRAD] = batched_kernel<FaceGradParams, face_grad_body, BW_THREADS, 1024>();
    table[KT_VERTEX_GRAD] = batched_kernel<VertexGradParams, vertex_grad_body, BW_THREADS, 1024>();
}

}  // namespace dc
