// server.cpp -- continuous-batching fit server (see cwb.h).
#include "runtime.h"

using namespace cwb;

extern "C" {
int cwb_server_create(const cwb_server_cfg*, cwb_server** out) {
  if (out) *out = nullptr;
  return set_error(CWB_E_UNSUPPORTED, "server not built yet");
}
int cwb_server_submit(cwb_server*, const cwb_problem*, uint64_t*) {
  return set_error(CWB_E_UNSUPPORTED, "server not built yet");
}
int cwb_server_poll(cwb_server*, uint64_t, cwb_result*, float*, int32_t*) {
  return set_error(CWB_E_UNSUPPORTED, "server not built yet");
}
int cwb_server_stats(cwb_server*, cwb_stats*) {
  return set_error(CWB_E_UNSUPPORTED, "server not built yet");
}
void cwb_server_destroy(cwb_server*) {}
}
