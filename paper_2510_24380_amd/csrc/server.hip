// Serving loop (continuous batching over one engine).
#include "engine_impl.h"

using namespace apex;

extern "C" apex_status apex_server_create(apex_engine*, const apex_server_config*, apex_server** out) {
  if (out) *out = nullptr;
  return set_error(APEX_E_UNSUPPORTED, "server not available in this build");
}
extern "C" apex_status apex_server_submit(apex_server*, const apex_query*, uint64_t*) {
  return set_error(APEX_E_UNSUPPORTED, "server not available in this build");
}
extern "C" apex_status apex_server_poll(apex_server*, uint64_t, apex_result*, int) {
  return set_error(APEX_E_UNSUPPORTED, "server not available in this build");
}
extern "C" apex_status apex_server_cancel(apex_server*, uint64_t) {
  return set_error(APEX_E_UNSUPPORTED, "server not available in this build");
}
extern "C" apex_status apex_server_stats_get(apex_server*, apex_server_stats*) {
  return set_error(APEX_E_UNSUPPORTED, "server not available in this build");
}
extern "C" apex_status apex_server_destroy(apex_server*) { return APEX_OK; }
