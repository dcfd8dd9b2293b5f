// Rigid bodies (Sec. III-C): a mesh vertex with body-frame coordinate p0 sits at
// p = [r] p0 + t for the 6-DoF pose q = (t_x, t_y, t_z, phi, theta, psi), with [r] read as
// Rz(psi) Ry(theta) Rx(phi).  Body b owns the vertices [body_start[b], body_start[b+1]).
//
//   k_rigid_fwd  one workgroup per (body, frame): the rotation in double, then every vertex of
//                the body in double, rounded once to float;
//   k_rigid_bwd  one workgroup per (body, frame): the pose gradient J^T g summed over the body's
//                vertices.  With G = sum_v g_v and S = sum_v g_v p0_v^T (twelve double sums, a
//                fixed-order tree over the workgroup), dL/dt = G and
//                dL/dr_k = sum_ij (dR/dr_k)_ij S_ij, since g . (dR p0) = <dR, g p0^T>.
// No atomics: every sum runs in a fixed order, so the result is bitwise reproducible.
#include "dc_internal.h"

namespace dc {
namespace {

constexpr int RG_THREADS = 256;

__device__ void mat3_mul(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// R = Rz(psi) Ry(theta) Rx(phi) and its partial derivatives in phi, theta, psi (row-major)
__device__ void pose_rotation(const double *qb, double *R, double *dR) {
    double sf, cf, st, ct, sp, cp;
    sincos(qb[3], &sf, &cf);
    sincos(qb[4], &st, &ct);
    sincos(qb[5], &sp, &cp);
    const double Rx[9] = {1, 0, 0, 0, cf, -sf, 0, sf, cf};
    const double Ry[9] = {ct, 0, st, 0, 1, 0, -st, 0, ct};
    const double Rz[9] = {cp, -sp, 0, sp, cp, 0, 0, 0, 1};
    const double dRx[9] = {0, 0, 0, 0, -sf, -cf, 0, cf, -sf};
    const double dRy[9] = {-st, 0, ct, 0, 0, 0, -ct, 0, -st};
    const double dRz[9] = {-sp, -cp, 0, cp, -sp, 0, 0, 0, 0};
    double M[9];
    mat3_mul(Rz, Ry, M);
    mat3_mul(M, Rx, R);
    if (!dR) return;
    mat3_mul(M, dRx, dR);
    mat3_mul(Rz, dRy, M);
    mat3_mul(M, Rx, dR + 9);
    mat3_mul(dRz, Ry, M);
    mat3_mul(M, Rx, dR + 18);
}

// the body's vertex range, or false (and the status bit) when it does not lie in [0, V]
__device__ __forceinline__ bool body_range(const int32_t *starts, int b, int V, unsigned *status,
                                           int &s, int &e) {
    s = starts[b];
    e = starts[b + 1];
    if (s < 0 || s > e || e > V) {
        if (threadIdx.x == 0 && blockIdx.y == 0) atomicOr(status, (unsigned)ST_BAD_INDEX);
        return false;
    }
    return true;
}

__global__ __launch_bounds__(RG_THREADS) void k_rigid_fwd(const double *__restrict__ q,
                                                          const float *__restrict__ p0,
                                                          const int32_t *__restrict__ starts,
                                                          int B, int V, float *__restrict__ verts,
                                                          unsigned *status) {
    const int b = blockIdx.x, t = blockIdx.y;
    int s, e;
    if (!body_range(starts, b, V, status, s, e)) return;
    const double *qb = q + ((size_t)t * B + b) * 6;
    double R[9];
    pose_rotation(qb, R, nullptr);
    for (int v = s + threadIdx.x; v < e; v += RG_THREADS) {
        const double x = p0[3 * (size_t)v], y = p0[3 * (size_t)v + 1], z = p0[3 * (size_t)v + 2];
        float *o = verts + ((size_t)t * V + v) * 3;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            o[i] = (float)(qb[i] + (R[3 * i] * x + R[3 * i + 1] * y + R[3 * i + 2] * z));
    }
}

__global__ __launch_bounds__(RG_THREADS) void k_rigid_bwd(const double *__restrict__ q,
                                                          const float *__restrict__ p0,
                                                          const int32_t *__restrict__ starts,
                                                          const float *__restrict__ gverts,
                                                          int B, int V, double *__restrict__ gq,
                                                          unsigned *status) {
    __shared__ double red[12][RG_THREADS];
    const int b = blockIdx.x, t = blockIdx.y;
    int s, e;
    if (!body_range(starts, b, V, status, s, e)) return;  // uniform over the workgroup
    double acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
    for (int v = s + threadIdx.x; v < e; v += RG_THREADS) {
        const float *g = gverts + ((size_t)t * V + v) * 3;
        const double p[3] = {p0[3 * (size_t)v], p0[3 * (size_t)v + 1], p0[3 * (size_t)v + 2]};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double gi = g[i];
            acc[i] += gi;
#pragma unroll
            for (int j = 0; j < 3; ++j) acc[3 + 3 * i + j] += gi * p[j];
        }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = RG_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int k = 0; k < 12; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double *qb = q + ((size_t)t * B + b) * 6;
        double R[9], dR[27];
        pose_rotation(qb, R, dR);
        double *o = gq + ((size_t)t * B + b) * 6;
        for (int i = 0; i < 3; ++i) o[i] = red[i][0];
        for (int a = 0; a < 3; ++a) {
            double d = 0.0;
            for (int ij = 0; ij < 9; ++ij) d += dR[9 * a + ij] * red[3 + ij][0];
            o[3 + a] = d;
        }
    }
}

}  // namespace

void launch_rigid_fwd(const double *q, const float *p0, const int32_t *body_start, int T, int B,
                      int V, float *verts, unsigned *status, hipStream_t s) {
    hipLaunchKernelGGL(k_rigid_fwd, dim3(B, T), dim3(RG_THREADS), 0, s, q, p0, body_start, B, V,
                       verts, status);
}

void launch_rigid_bwd(const double *q, const float *p0, const int32_t *body_start,
                      const float *grad_verts, int T, int B, int V, double *grad_q,
                      unsigned *status, hipStream_t s) {
    hipLaunchKernelGGL(k_rigid_bwd, dim3(B, T), dim3(RG_THREADS), 0, s, q, p0, body_start,
                       grad_verts, B, V, grad_q, status);
}

}  // namespace dc
