// Serving loop of libdiffcloud: dc_submit / dc_poll / dc_wait.
#pragma once

#include "dc_internal.h"

namespace dc {

int sched_submit(dc_ctx *ctx, const dc_request *req, dc_result *out, uint64_t *ticket);
int sched_poll(dc_ctx *ctx, uint64_t ticket);
int sched_wait(dc_ctx *ctx, uint64_t ticket, long long timeout_us);
void sched_destroy(dc_ctx *ctx);

// device bytes a request holds while admitted (inputs, intermediates, outputs, scratch)
size_t request_bytes(int T, int V, int F, int Na, int Nb, int precision, bool want_grad);

}  // namespace dc
