// Internal declarations of libdiffcloud: context, scratch arena, error state, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/diffcloud.h"

namespace dc {

// ---------------------------------------------------------------- error state
void set_error(const std::string &msg);
void clear_error();
int hip_fail(hipError_t e, const char *what);  // records the message, returns DC_ERR_HIP

#define DC_HIP(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return ::dc::hip_fail(e_, #call); \
    } while (0)

// bits of the sticky device status word
enum : unsigned { ST_DEGENERATE = 1u, ST_BAD_FACE = 2u, ST_BAD_INDEX = 4u };

// ---------------------------------------------------------------- scratch arena
// A grow-only device buffer carved into 256-byte aligned pieces per call.  Growing frees the old
// buffer only after the device is idle, so work still in flight never loses its memory.
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t off = 0;
    void reset() { off = 0; }
    template <class T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base + off);
        off += bytes;
        return p;
    }
    static size_t need(size_t count, size_t elem) { return (count * elem + 255) & ~size_t(255); }
};

struct Scheduler;

// events bracketing profiled launches: (category, start, stop)
struct ProfRecord {
    int cat;
    hipEvent_t a, b;
};

}  // namespace dc

struct dc_ctx {
    int device = 0;
    size_t budget = 0;
    int max_slots = 64;
    std::mutex mu;                // serialises direct calls (they share the arena)
    std::mutex budget_mu;         // guards budget accounting
    size_t held = 0;              // bytes of device memory held against the budget
    dc::Arena arena;              // scratch of direct calls
    hipEvent_t arena_ev = nullptr;        // recorded after each direct call's work on its stream
    hipStream_t arena_stream = nullptr;   // the stream of the last direct call
    bool arena_used = false;
    unsigned *d_status = nullptr;           // sticky device status word
    unsigned long long *d_stats = nullptr;  // screen counters: [STATS_SLOTS][STATS_SLOT_WORDS]
    dc::Scheduler *sched = nullptr;
    int fail_next_alloc = 0;      // test hook: make the next N allocations fail
    bool prof = false;            // record events around profiled launches
    std::mutex prof_mu;
    std::vector<dc::ProfRecord> prof_pending;
    double prof_ms[4] = {0, 0, 0, 0};
    uint64_t prof_n[4] = {0, 0, 0, 0};
};

namespace dc {

// reserve `bytes` of the budget; DC_ERR_BUDGET if it cannot fit
int budget_take(dc_ctx *ctx, size_t bytes);
void budget_give(dc_ctx *ctx, size_t bytes);
// The screen's counters (queries, candidate groups, fallbacks) are spread over STATS_SLOTS slots of
// STATS_SLOT_WORDS 64-bit words (one 128-byte cache line per slot); a workgroup adds its counts to
// the slot of its hardware id and the host sums the slots.  One shared counter would serialise
// the atomics of every workgroup on one address.
constexpr int STATS_SLOTS = 64;
constexpr int STATS_SLOT_WORDS = 16;
constexpr size_t STATS_BYTES = sizeof(unsigned long long) * STATS_SLOTS * STATS_SLOT_WORDS;
// device bytes of the context's status and counter words (held from dc_create on)
constexpr size_t CTX_WORDS_BYTES = sizeof(unsigned) * 4 + STATS_BYTES;
// test hook: true (and one fewer pending) when the next allocation is to fail
bool forced_alloc_failure(dc_ctx *ctx);
// device allocation counted against the budget; dev_alloc honours the test hook, dev_alloc_raw
// does not (its caller has consulted the hook for the allocation it serves)
int dev_alloc(dc_ctx *ctx, void **p, size_t bytes);
int dev_alloc_raw(dc_ctx *ctx, void **p, size_t bytes);
void dev_free(dc_ctx *ctx, void *p, size_t bytes);
// Make sure the direct-call arena holds at least `bytes` and reset its offset.  When the previous
// direct call ran on another stream, `s` first waits for that call's work, so calls on different
// streams never share the scratch in time.
int arena_reserve(dc_ctx *ctx, size_t bytes, hipStream_t s);
// mark the end of a direct call's use of the arena (records the arena event on `s`)
struct ArenaUse {
    dc_ctx *ctx;
    hipStream_t s;
    ~ArenaUse();
};

// start / stop an event pair around the launches of category `cat` (no-op unless profiling)
struct ProfScope {
    dc_ctx *ctx;
    int cat;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(dc_ctx *c, int category, hipStream_t st);
    ~ProfScope();
};

// ---------------------------------------------------------------- launchers (async, on `s`)
// sampling
size_t sample_scratch_bytes(int T, int F);
// the per-frame face areas and their running sum (cdf [T,F] double, lastpos [T]: last face of
// positive area, -1 for a degenerate frame or one with an invalid face)
void launch_area_cdf(const float *verts, const int32_t *faces, int T, int V, int F,
                     const uint8_t *mask, int mask_per_frame, double *cdf, int32_t *lastpos,
                     unsigned *status, hipStream_t s);
void launch_sample(const float *verts, const int32_t *faces, int T, int V, int F, int N,
                   uint64_t seed, const uint32_t *uniforms, const uint8_t *mask, int mask_per_frame,
                   float *points, int32_t *face_idx, float *bary, double *cdf_scratch,
                   int32_t *lastpos_scratch, unsigned *status, hipStream_t s);

// exact fp32 nearest neighbours: for each query of Q[t] the index of its nearest point in P[t]
size_t nn_exact_scratch_bytes(int T, int Nq, int Np);
void launch_nn_exact_ws(const float *Q, int Nq, const float *P, int Np, int T, int32_t *idx,
                        float *dist, char *scratch, hipStream_t st);
// both directions in one pass (each pair evaluated once), when the frames have enough rows to
// fill the chip; false (nothing launched) otherwise
size_t nn_bidir_scratch_bytes(int T, int Na, int Nb);
bool launch_nn_bidir(const float *A, int Na, const float *B, int Nb, int T, int32_t *idx_a,
                     float *dist_a, int32_t *idx_b, float *dist_b, char *scratch, hipStream_t st);
// the same search restricted, per frame t, to the rows qlist[t*Nq + k], k < qcount[t]
size_t nn_exact_list_scratch_bytes(int T, int Nq, int Np);
void launch_nn_exact_list(const float *Q, int Nq, const float *P, int Np, int T,
                          const int32_t *qlist, const int32_t *qcount, int32_t *idx, float *dist,
                          char *scratch, hipStream_t st);

// bf16 matrix-core screen + certified exact refine, both directions in one pass (the same
// indices and distances as two exact fp32 searches)
size_t screen_scratch_bytes(int T, int Na, int Nb);
void launch_chamfer_screened(const float *a, int Na, const float *b, int Nb, int T,
                             int32_t *idx_a, float *dist_a, int32_t *idx_b, float *dist_b,
                             char *scratch, unsigned long long *stats, dc_ctx *prof,
                             hipStream_t s);

// per-frame loss from the float distances, accumulated in double
void launch_loss(const float *dist_a, const float *dist_b, int T, int Na, int Nb, int reduction,
                 const float *frame_w, double *loss, hipStream_t s);

// stable, atomic-free sort of per-frame keys in [0, key_limit]: out_keys/out_vals get the keys
// and the original positions in (key, position) order.  Keys outside the range sort as key_limit;
// with mark_invalid their value is the complement of their position (negative).
size_t segsort_scratch_bytes(int T, int N);
void launch_segsort(const int32_t *keys, int T, int N, int key_limit, int32_t *out_keys,
                    int32_t *out_vals, char *scratch, hipStream_t s, bool mark_invalid = false);

// Chamfer backward
size_t chamfer_bwd_scratch_bytes(int T, int Na, int Nb, bool want_b);
void launch_chamfer_bwd(const double *grad_loss, const float *a, const float *b,
                        const int32_t *idx_a, const int32_t *idx_b, int T, int Na, int Nb,
                        int reduction, const float *frame_w, float *grad_a, float *grad_b,
                        char *scratch, hipStream_t s);

// sampling backward
size_t sample_bwd_scratch_bytes(int T, int V, int F, int N);
void launch_sample_bwd(const float *grad_points, const int32_t *faces, const int32_t *face_idx,
                       const float *bary, int T, int V, int F, int N, float *grad_verts,
                       char *scratch, hipStream_t s);

// rigid bodies: vertices from 6-DoF poses, and the pose gradient
void launch_rigid_fwd(const double *q, const float *p0, const int32_t *body_start, int T, int B,
                      int V, float *verts, unsigned *status, hipStream_t s);
void launch_rigid_bwd(const double *q, const float *p0, const int32_t *body_start,
                      const float *grad_verts, int T, int B, int V, double *grad_q,
                      unsigned *status, hipStream_t s);

// the allocation-free sampling entry point: look up its scratch address on `device` (once per
// device, with that device current)
int noalloc_init(int device);

// composite enqueues shared by the direct calls and the serving loop
// `prof` is the context whose profiling records the launches, or NULL
int enqueue_sample(dc_ctx *prof, const float *verts, const int32_t *faces, int T, int V, int F,
                   int N, uint64_t seed, const uint32_t *uniforms, const uint8_t *mask,
                   int mask_per_frame, float *points, int32_t *face_idx, float *bary, Arena &ar,
                   unsigned *status, hipStream_t s);
size_t chamfer_fwd_scratch_bytes(int T, int Na, int Nb, int precision);
int enqueue_chamfer_fwd(dc_ctx *prof, const float *a, const float *b, int T, int Na, int Nb,
                        int precision,
                        int reduction, const float *frame_w, float *dist_a, int32_t *idx_a,
                        float *dist_b, int32_t *idx_b, double *loss, char *scratch,
                        unsigned long long *stats, hipStream_t s);

}  // namespace dc
