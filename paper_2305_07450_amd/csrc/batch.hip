// batch.hip - batched persistent launch (not built yet: every entry point
// reports RT_ERR_UNSUPPORTED).
#include "rt_internal.hpp"

using namespace rtk;

extern "C" {

rt_status rt_batch_create(int32_t, const rt_scene*, const rt_camera*, const int32_t*,
                          const int32_t*, const int32_t*, float* const*, int32_t, void*,
                          rt_batch* out) {
  if (out) *out = nullptr;
  set_error("rt_batch_create is not available in this build");
  return RT_ERR_UNSUPPORTED;
}
rt_status rt_batch_launch(rt_batch, void*) {
  set_error("rt_batch_launch is not available in this build");
  return RT_ERR_UNSUPPORTED;
}
rt_status rt_batch_launch_direct(rt_batch, void*) {
  set_error("rt_batch_launch_direct is not available in this build");
  return RT_ERR_UNSUPPORTED;
}
rt_status rt_batch_shape(rt_batch, int32_t*, int32_t*, int32_t*) {
  set_error("rt_batch_shape is not available in this build");
  return RT_ERR_UNSUPPORTED;
}
rt_status rt_batch_destroy(rt_batch) { return RT_OK; }

}  // extern "C"
