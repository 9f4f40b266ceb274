// Serving loop (placeholder until the request engine is built).
#include "internal.h"

extern "C" {
tc_status tc_serve_create(const tc_serve_opts*, tc_server**) {
  tcx::set_error("serving not built");
  return TC_ERR_UNSUPPORTED;
}
tc_status tc_serve_submit(tc_server*, const tc_circuit*, const tc_observable*, const float*,
                          int32_t, int64_t*) {
  tcx::set_error("serving not built");
  return TC_ERR_UNSUPPORTED;
}
tc_status tc_serve_step(tc_server*, int32_t*) {
  tcx::set_error("serving not built");
  return TC_ERR_UNSUPPORTED;
}
tc_status tc_serve_result_get(tc_server*, int64_t, tc_serve_result*, double*) {
  tcx::set_error("serving not built");
  return TC_ERR_UNSUPPORTED;
}
void tc_serve_free(tc_server*) {}
}
