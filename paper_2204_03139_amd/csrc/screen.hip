// bf16 matrix-core screen with certified exact refine: not built yet in this revision.
#include "dc_internal.h"

namespace dc {

bool screen_available() { return false; }

size_t screen_scratch_bytes(int, int, int) { return 0; }

void launch_nn_screened(const float *, int, const float *, int, int, int32_t *, float *, char *,
                        unsigned long long *, dc_ctx *, hipStream_t) {}

}  // namespace dc
