// Entry points whose kernels are not written yet: they report MELT_E_UNSUPPORTED.
#include "melt_internal.h"

namespace melt {
melt_status launch_melt_backward(Plan &, const float *, const int64_t *, int, int64_t, const float *, const float *,
                                 float *, float *, hipStream_t) {
    return set_error(MELT_E_UNSUPPORTED, "melt_backward not built");
}
}  // namespace melt

extern "C" {
melt_status melt_stream_create(melt_plan, int32_t, int32_t, melt_stream_state *) { return MELT_E_UNSUPPORTED; }
melt_status melt_stream_destroy(melt_stream_state) { return MELT_OK; }
melt_status melt_stream_reset(melt_stream_state, void *) { return MELT_E_UNSUPPORTED; }
int32_t melt_stream_max_frames(melt_stream_state) { return 0; }
melt_status melt_stream_push(melt_stream_state, const float *, float *, int32_t *, void *) { return MELT_E_UNSUPPORTED; }
melt_status melt_autotune(melt_plan, int64_t, char *, int32_t) { return MELT_E_UNSUPPORTED; }
}
