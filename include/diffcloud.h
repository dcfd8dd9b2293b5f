/*
 * diffcloud.h - C ABI of the MI355X (gfx950) DiffCloud hot-path library, libdiffcloud.so.
 *
 * The library computes, on one GPU, the data-parallel part of the DiffCloud gradient pipeline
 * (arXiv 2204.03139): area-weighted point sampling from triangle-mesh trajectories
 * (Sec. III-B, Eq. 3), the bidirectional or unidirectional Chamfer distance to an observed cloud
 * (Sec. III-A, Eq. 1 and Eq. 2), and the backward pass to per-vertex gradients through Eq. 4,
 * for every frame of a trajectory (Sec. III-C).
 *
 * Conventions shared by every entry point
 *  - All arrays are dense, row-major, little-endian.  Coordinates are float32 triples (x, y, z).
 *    [T,N,3] means frame-major: element (t, i, k) sits at ((t*N)+i)*3+k.
 *  - Pointers marked "device" must be device memory of the context's GPU (for example a torch
 *    tensor's data_ptr()).  The caller owns them; the library never frees or keeps them past the
 *    call's stream work.  Pointers marked "host" are ordinary host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Direct calls are
 *    asynchronous: they validate their arguments on the host, enqueue kernels on `stream` and
 *    return.  Calls that share one context share its scratch memory: a call on a different stream
 *    than the previous call of the context first makes its stream wait (on the device) for the
 *    previous call's work, so such calls never overlap in time.  The caller still orders its own
 *    data dependences between streams.
 *  - Every entry point returns a status code.  No exception crosses the ABI.  Argument errors are
 *    reported immediately.  Errors that only the device can see (a face index outside [0, V), a
 *    frame whose total area is zero or not finite) set a sticky status word in the context, and
 *    dc_sync() reports and clears it.  The text of the last error of the calling thread is
 *    available from dc_last_error().
 *  - Limits: 1 <= T <= 65535; 1 <= N, Na, Nb, V, F <= 2^24.  NaN or infinite coordinates are not
 *    validated; they propagate and the neighbour indices they produce are unspecified.
 */
#ifndef DIFFCLOUD_H
#define DIFFCLOUD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define DC_OK 0
#define DC_PENDING 1           /* dc_poll: the request is queued or running */
#define DC_ERR_INVALID (-1)    /* bad argument (null pointer, size out of range, bad enum) */
#define DC_ERR_NOMEM (-2)      /* a device allocation failed */
#define DC_ERR_BUDGET (-3)     /* the work can never fit the context's HBM budget */
#define DC_ERR_HIP (-4)        /* a HIP runtime call failed; see dc_last_error() */
#define DC_ERR_DEGENERATE (-5) /* a frame's total surface area is zero or not finite */
#define DC_ERR_UNSUPPORTED (-6)/* a valid request the library cannot run (serving program) */

/* precision of the all-pairs nearest-neighbour search (both give the same indices) */
#define DC_PREC_FP32 0        /* exact single-precision search on the vector ALUs */
#define DC_PREC_BF16_REFINE 1 /* bf16 matrix-core screen, certified, exact fp32 re-evaluation */

/* reduction of the two directions into the per-frame loss */
#define DC_RED_BIDIR_MEAN 0   /* Eq. 1: mean over a of min_b + mean over b of min_a */
#define DC_RED_SIM2REAL_SUM 1 /* Eq. 2: sum over a (simulated) of min over b (observed) */

typedef struct dc_ctx dc_ctx;

/* ------------------------------------------------------------------ context */
/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device memory the context
 * holds at any time (0 means 64 GiB): its status words, the scratch of direct calls (grow-only,
 * kept until dc_destroy), and once the serving loop has started, its batch descriptors and the
 * segments its requests' regions are carved from (kept while requests are in flight, given back
 * only when none is).  max_slots caps the requests the serving loop keeps in flight (0 means 64).
 * On success *out receives the context.
 * Errors: DC_ERR_INVALID, DC_ERR_HIP, DC_ERR_NOMEM, DC_ERR_BUDGET (budget below a few hundred
 * bytes). */
int dc_create(dc_ctx **out, int device, size_t hbm_budget_bytes, int max_slots);

/* Wait for the serving loop to drain, free everything the context owns, destroy it.  No other
 * call on the context may be in progress (a thread blocked in dc_wait included) or follow: the
 * caller collects its requests' results first. */
int dc_destroy(dc_ctx *ctx);

/* Text of the calling thread's last error ("" if none); valid until the thread's next call into
 * the library.  Messages are kept per thread, not per context: `ctx` may be NULL and is not read
 * (it is part of the signature so that a caller can name the context it is asking about). */
const char *dc_last_error(const dc_ctx *ctx);

/* Wait for `stream`, then report and clear device-detected errors of earlier direct calls:
 * DC_OK, DC_ERR_DEGENERATE (a frame with zero or non-finite total area; its points are NaN and
 * its face indices -1) or DC_ERR_INVALID (a face index outside [0, V)). */
int dc_sync(dc_ctx *ctx, void *stream);

/* ------------------------------------------------------------------ sampling, Sec. III-B */
/* Draw N points per frame on the surface of the mesh (verts[t], faces), Eq. 3.
 *   verts    device float [T,V,3]   vertex positions per frame
 *   faces    device int32 [F,3]     corner vertex indices, the same for every frame
 *   seed     key of the counter-based generator, used when uniforms is NULL
 *   uniforms device uint32 [T,N,4] or NULL: four random words per (frame, point)
 *   points   device float [T,N,3]   out: sampled points
 *   face_idx device int32 [T,N]     out: face of each point
 *   bary     device float [T,N,3]   out: (u, v, w) of each point
 * Arithmetic, per frame t:
 *   A_f  = |(p2-p1) x (p3-p1)| / 2 in double from the float corners (no fused operations);
 *   C_k  = C_{k-1} + A_k in double, left to right; S = C_{F-1};
 *   face = first k with C_k > r*S, r = (53 high bits of words 0,1) * 2^-53 (word 1 is the high
 *          half); if none, the last face with A_k > 0; zero-area faces are never drawn;
 *   r1, r2 = (word >> 8) * 2^-24 of words 2 and 3; s = correctly rounded sqrt(r1);
 *   u = 1-s, v = s(1-r2), w = s r2 (the square-root construction of Osada et al. 2002);
 *   x = fma(w, p3, fma(v, p2, u*p1)) per coordinate, in float.
 * With uniforms == NULL the words come from Philox4x64-10 (Salmon et al., SC'11) with counter
 * (i, t, 0, 0) and key (seed, 0): words 0,1 = low, high half of output 0; word 2 = high half of
 * output 1; word 3 = high half of output 2.
 * Errors: DC_ERR_INVALID (argument), DC_ERR_HIP; zero or non-finite total area and bad face
 * indices are reported by dc_sync(). */
int dc_sample_surface(dc_ctx *ctx, const float *verts, const int32_t *faces, int T, int V, int F,
                      int N, uint64_t seed, const uint32_t *uniforms, float *points,
                      int32_t *face_idx, float *bary, void *stream);

/* dc_sample_surface restricted to a subset of the faces (the subset sampling of Sec. IV: the
 * occlusion heuristic that samples only the visible part of the cloth, cloth-only clouds of a
 * scene, biased subsets that mimic partial observations).
 *   face_mask      device uint8, nonzero = the face may be drawn: [F] shared by all frames
 *                  (mask_per_frame = 0) or [T,F] one row per frame (mask_per_frame = 1)
 * A face outside the subset takes part with A_f = 0 in the running sum, so it is never drawn and
 * the other faces keep their area weights; everything else is as in dc_sample_surface.  A frame
 * whose subset has zero total area is reported by dc_sync() like any degenerate frame.
 * Errors: as dc_sample_surface; DC_ERR_INVALID also for a NULL mask or mask_per_frame not 0/1. */
int dc_sample_surface_masked(dc_ctx *ctx, const float *verts, const int32_t *faces, int T, int V,
                             int F, int N, uint64_t seed, const uint32_t *uniforms,
                             const uint8_t *face_mask, int mask_per_frame, float *points,
                             int32_t *face_idx, float *bary, void *stream);

/* The first two steps of dc_sample_surface on their own: the face areas and their running sum,
 * the inverse-CDF table that Eq. 3's area-weighted choice of a face is drawn from (Sec. III-B).
 *   verts, faces, T, V, F   as dc_sample_surface
 *   face_mask  device uint8 [F] (mask_per_frame = 0) or [T,F] (mask_per_frame = 1), or NULL (all
 *              faces): as dc_sample_surface_masked, a face outside the subset has A_f = 0
 *   cdf        device double [T,F] out: C_k = C_{k-1} + A_k, left to right from C_{-1} = 0, each
 *              sum rounded to double - bit for bit the plain sequential sum of the A_f, which are
 *              computed exactly as in dc_sample_surface
 *   last_face  device int32 [T] or NULL; out: the last face with A_k > 0 (the face drawn when
 *              rounding leaves no C_k above r*S), -1 for a frame whose total is zero or not
 *              finite or whose faces name a vertex outside [0, V)
 * Errors: DC_ERR_INVALID (argument, or mask_per_frame not 0/1), DC_ERR_HIP, DC_ERR_NOMEM,
 * DC_ERR_BUDGET; zero or non-finite totals and bad face indices are reported by dc_sync(), as for
 * dc_sample_surface. */
int dc_area_cdf(dc_ctx *ctx, const float *verts, const int32_t *faces, int T, int V, int F,
                const uint8_t *face_mask, int mask_per_frame, double *cdf, int32_t *last_face,
                void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): dc_sample_surface with the same arguments, arithmetic,
 * results and errors, except that its scratch - the per-frame area CDF in double and the last
 * drawable face of each frame, T*F*8 + T*4 bytes, each part rounded up to 256 - lives in a static
 * device array of 16 MiB per GPU instead of the context's scratch, so the call allocates nothing
 * (the context's own memory is untouched).  The array exists on every GPU the library runs on and
 * is held until the process ends.  T and F whose scratch exceeds 16 MiB (T*F above about 2.09
 * million; 100 frames of 19,602 faces fit) give DC_ERR_UNSUPPORTED.  Every call on one GPU shares
 * its array, which keeps the last call's contents: calls whose device work overlaps (on different
 * streams, or from different contexts of the same GPU) race, so order them on one stream or with
 * events. */
int dc_sample_surface_noalloc(dc_ctx *ctx, const float *verts, const int32_t *faces, int T, int V,
                              int F, int N, uint64_t seed, const uint32_t *uniforms,
                              float *points, int32_t *face_idx, float *bary, void *stream);

/* Backward of dc_sample_surface through Eq. 4 (dx_i/dp_{i,c} = bary_c(i) I):
 *   grad_verts[t,v] = sum over points i of frame t and corners c with faces[face_idx[t,i]][c]==v
 *                     of bary[t,i,c] * grad_points[t,i].
 * No gradient flows through the face choice or the areas.  Sums run in a fixed order (by vertex
 * incidence, then by point index) and in double (each (face, corner) sum and each output rounded
 * once to float), so the result is bitwise reproducible; no atomics are used.
 *   grad_points device float [T,N,3]; faces, face_idx, bary as produced by dc_sample_surface;
 *   grad_verts  device float [T,V,3], overwritten.
 * Points whose face_idx is -1 (degenerate frame) contribute nothing.
 * Errors: DC_ERR_INVALID, DC_ERR_HIP, DC_ERR_NOMEM, DC_ERR_BUDGET (scratch over budget). */
int dc_sample_surface_bwd(dc_ctx *ctx, const float *grad_points, const int32_t *faces,
                          const int32_t *face_idx, const float *bary, int T, int V, int F, int N,
                          float *grad_verts, void *stream);

/* ------------------------------------------------------------------ Chamfer, Sec. III-A */
/* Nearest neighbours in both directions and the per-frame loss, Eq. 1 or Eq. 2.
 *   a, b      device float [T,Na,3], [T,Nb,3]   simulated (a) and observed (b) clouds
 *   precision DC_PREC_FP32 or DC_PREC_BF16_REFINE (same results; different speed)
 *   reduction DC_RED_BIDIR_MEAN (Eq. 1) or DC_RED_SIM2REAL_SUM (Eq. 2)
 *   frame_w   device float [T] or NULL (all ones): weight w_t of frame t
 *   dist_a, idx_a  device float/int32 [T,Na] out: min over b, and its index
 *   dist_b, idx_b  device float/int32 [T,Nb] out: min over a, and its index; with
 *             DC_RED_SIM2REAL_SUM both may be NULL (together): then only the a -> b direction
 *             is searched, which is all that Eq. 2 and its gradient to a need
 *   loss      device double [T] out: loss[t] = w_t (alpha sum_i dist_a + beta sum_j dist_b),
 *             alpha = 1/Na, beta = 1/Nb for Eq. 1; alpha = 1, beta = 0 for Eq. 2.
 * The neighbour of a point is decided by the canonical float squared distance
 *   d = fma(dz, dz, fma(dy, dy, dx*dx)), dx = ax - bx rounded to float,
 * ties going to the smallest index; dist_* hold that float d.  The loss sums the float distances
 * in double.
 * Errors: DC_ERR_INVALID (also: only one of dist_b / idx_b NULL, or NULL with Eq. 1), DC_ERR_HIP,
 * DC_ERR_NOMEM, DC_ERR_BUDGET. */
int dc_chamfer_fwd(dc_ctx *ctx, const float *a, const float *b, int T, int Na, int Nb,
                   int precision, int reduction, const float *frame_w, float *dist_a,
                   int32_t *idx_a, float *dist_b, int32_t *idx_b, double *loss, void *stream);

/* Backward of dc_chamfer_fwd with the neighbours of the forward held fixed (a subgradient at
 * ties), for the upstream gradient g_t = grad_loss[t] of loss[t]:
 *   grad_a[t,i] = g_t w_t ( 2 alpha (a_i - b_{idx_a[i]}) + 2 beta sum_{j: idx_b[j]=i} (a_i - b_j) )
 *   grad_b[t,j] = g_t w_t ( 2 beta (b_j - a_{idx_b[j]}) + 2 alpha sum_{i: idx_a[i]=j} (b_j - a_i) )
 * The sums over j (resp. i) run in increasing index order after a stable, atomic-free sort by
 * neighbour index, in double (each output rounded once to float), so results are bitwise
 * reproducible.  A neighbour index outside [0, Nb) (resp.
 * [0, Na)) contributes nothing: neither its own term nor a term to the point it names.
 *   grad_loss device double [T]; a, b, idx_a, idx_b, frame_w as in dc_chamfer_fwd (idx_b is not
 *   read with DC_RED_SIM2REAL_SUM, where beta = 0, and may then be NULL);
 *   grad_a device float [T,Na,3] out (overwritten); grad_b device float [T,Nb,3] or NULL.
 * Errors: DC_ERR_INVALID, DC_ERR_HIP, DC_ERR_NOMEM, DC_ERR_BUDGET. */
int dc_chamfer_bwd(dc_ctx *ctx, const double *grad_loss, const float *a, const float *b,
                   const int32_t *idx_a, const int32_t *idx_b, int T, int Na, int Nb,
                   int reduction, const float *frame_w, float *grad_a, float *grad_b,
                   void *stream);

/* ------------------------------------------------------------------ rigid bodies, Sec. III-C */
/* World vertices of rigid meshes from their 6-DoF poses: a vertex with body-frame coordinate p0
 * sits at p = [r] p0 + t, q = (t_x, t_y, t_z, phi, theta, psi), [r] = Rz(psi) Ry(theta) Rx(phi).
 *   q          device double [T,B,6]  pose of body b at frame t
 *   p0         device float [V,3]     body-frame coordinates
 *   body_start device int32 [B+1]     body b owns the vertices [body_start[b], body_start[b+1])
 *   verts      device float [T,V,3]   out: the bodies' vertices (computed in double, rounded once
 *              to float); vertices owned by no body are left untouched (deformables of a scene)
 * A range outside [0, V] or decreasing is reported by dc_sync() as DC_ERR_INVALID.
 * Errors: DC_ERR_INVALID (argument), DC_ERR_HIP. */
int dc_rigid_pose(dc_ctx *ctx, const double *q, const float *p0, const int32_t *body_start,
                  int T, int B, int V, float *verts, void *stream);

/* Chain rule from vertex gradients to the poses (the Jacobian of p = f(q), Sec. III-C):
 *   grad_q[t,b] = sum over the vertices v of body b of J_v^T grad_verts[t,v],
 *   J_v = [ I | dR/dphi p0_v | dR/dtheta p0_v | dR/dpsi p0_v ]  (3 x 6),
 * summed in double in a fixed order (bitwise reproducible, no atomics).
 *   grad_verts device float [T,V,3]; grad_q device double [T,B,6] out (overwritten).
 * Errors: as dc_rigid_pose. */
int dc_rigid_pose_bwd(dc_ctx *ctx, const double *q, const float *p0, const int32_t *body_start,
                      const float *grad_verts, int T, int B, int V, double *grad_q,
                      void *stream);

/* Counters of the bf16 screen since the context was created (read after dc_sync):
 *   queries    nearest-neighbour queries answered by the screened search
 *   candidates candidate groups re-evaluated exactly
 *   fallbacks  queries whose certificate failed and that were searched exhaustively */
typedef struct dc_stats {
    uint64_t queries;
    uint64_t candidates;
    uint64_t fallbacks;
} dc_stats;
int dc_get_stats(dc_ctx *ctx, dc_stats *out);

/* ------------------------------------------------------------------ kernel timing */
/* With profiling on, the direct calls bracket their kernels with HIP events on the caller's
 * stream and accumulate the elapsed device time per category:
 *   [0] the all-pairs nearest-neighbour kernel (exact fp32 search, or the bf16 screen)
 *   [1] the exact re-evaluation of screened candidates
 *   [2] sampling (areas, CDF, face choice, points)
 *   [3] the backward kernels (Chamfer and sampling backward, their sorts)
 * dc_get_kernel_times waits for the recorded events, returns the sums and launch counts, and
 * resets them when `reset` is nonzero.  Profiling costs two event records per launch. */
typedef struct dc_kernel_times {
    double ms[4];
    uint64_t launches[4];
} dc_kernel_times;
int dc_profile(dc_ctx *ctx, int enable);
int dc_get_kernel_times(dc_ctx *ctx, dc_kernel_times *out, int reset);

/* ------------------------------------------------------------------ serving loop */
/* One calibration query: a mesh trajectory, an observed cloud sequence, and how to compare
 * them.  All pointers are host memory, copied into context-owned device memory at admission;
 * the caller may reuse them as soon as dc_submit returns. */
typedef struct dc_request {
    const float *verts;    /* host float [T,V,3] */
    const int32_t *faces;  /* host int32 [F,3] */
    int T, V, F;
    int n_sim;             /* points sampled per frame (Na) */
    const float *observed; /* host float [T,n_obs,3] */
    int n_obs;             /* observed points per frame (Nb) */
    uint64_t seed;         /* sampler key (the uniforms come from the counter-based generator) */
    int precision;         /* DC_PREC_* */
    int reduction;         /* DC_RED_* */
    const float *frame_w;  /* host float [T] or NULL */
} dc_request;

/* Result of a request, written by the library; the caller owns it and must keep it alive until
 * dc_poll() returns something other than DC_PENDING for its ticket. */
typedef struct dc_result {
    double *loss;       /* host double [T], caller-allocated; out: loss[t] */
    float *grad_verts;  /* host float [T,V,3] caller-allocated, or NULL; out: d(sum_t loss[t])/dV */
    double t_submit;    /* seconds (steady clock) when dc_submit accepted the request */
    double t_admit;     /* when its device memory was granted and its work enqueued */
    double t_done;      /* when its results were on the host */
    int status;         /* DC_OK or an error code once done */
} dc_result;

/* Queue a request.  Its host inputs are copied into pinned staging before the call returns.
 * Requests are admitted in arrival order, each once a device region of dc_request_bytes() can be
 * carved from the serving loop's memory (growing it if the budget allows) and fewer than
 * max_slots requests are in flight; admitted requests are batched with whatever else is waiting
 * and run on the device alongside requests already in flight.  A request that cannot fit waits
 * while others are in flight; if it still cannot fit when none is (the direct calls' scratch
 * holds too much of the budget), it fails with DC_ERR_BUDGET, and a refused device allocation
 * fails it with DC_ERR_NOMEM: either way alone, the others of its batch are unaffected.  A
 * request larger than the budget can ever hold (its region beside the context's status words and
 * the serving loop's batch descriptors, about 1.1 MB) fails with DC_ERR_BUDGET at once.  *ticket
 * identifies it for dc_poll().  Thread-safe. */
int dc_submit(dc_ctx *ctx, const dc_request *req, dc_result *out, uint64_t *ticket);

/* Device bytes the request would hold while admitted (inputs, intermediates, outputs, scratch),
 * the amount admission reserves against the budget.  want_grad selects whether the backward runs
 * (dc_submit runs it when the result's grad_verts is not NULL).  Errors: DC_ERR_INVALID. */
int dc_request_bytes(const dc_request *req, int want_grad, size_t *bytes);

/* DC_PENDING while queued or running.  Once the request has finished, the poll copies its
 * results into the caller's dc_result buffers, sets status and t_done, and returns the final
 * status (DC_OK or an error); the ticket is then forgotten (a second poll gives DC_ERR_INVALID).
 * Thread-safe. */
int dc_poll(dc_ctx *ctx, uint64_t ticket);

/* dc_poll that first waits for the request to finish: up to timeout_us microseconds (a negative
 * value: without limit), sleeping until the serving loop marks a request done rather than
 * polling.  Returns DC_PENDING if the request is still queued or running when the time is up;
 * otherwise exactly what dc_poll returns, with the results handed over in the same way.  One
 * thread should wait on or poll a given ticket; any number of threads may wait on different
 * tickets.  Thread-safe. */
int dc_wait(dc_ctx *ctx, uint64_t ticket, int64_t timeout_us);

/* Device bytes the context holds against its budget now (*held), and the budget (*budget, may be
 * NULL).  Errors: DC_ERR_INVALID. */
int dc_memory_held(dc_ctx *ctx, size_t *held, size_t *budget);

/* Test hook: make the context's next n device allocations fail with DC_ERR_NOMEM, so that
 * failure handling can be exercised without exhausting the device.  An allocation is a growth of
 * the direct calls' scratch, or the device region of one serving request at its admission (that
 * request then fails alone). */
int dc_debug_fail_allocs(dc_ctx *ctx, int n);

/* Library version as major*10000 + minor*100 + patch. */
int dc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DIFFCLOUD_H */
