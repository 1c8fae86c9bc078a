// Serving loop (continuous batching) over a resident background summary.
#include "wdf_impl.h"

extern "C" int wdf_server_create(const wdf_bg *, size_t, int, int, wdf_server **out) {
  if (out) *out = nullptr;
  return wdf::set_error(WDF_E_UNSUPPORTED, "wdf_server_create: not available yet");
}
extern "C" int wdf_server_submit(wdf_server *, const float *, int64_t, int64_t, float *, uint64_t *) {
  return wdf::set_error(WDF_E_UNSUPPORTED, "wdf_server_submit: not available yet");
}
extern "C" int wdf_server_wait(wdf_server *, uint64_t, int) {
  return wdf::set_error(WDF_E_UNSUPPORTED, "wdf_server_wait: not available yet");
}
extern "C" int wdf_server_stats(wdf_server *, wdf_stats *) {
  return wdf::set_error(WDF_E_UNSUPPORTED, "wdf_server_stats: not available yet");
}
extern "C" void wdf_server_destroy(wdf_server *) {}
