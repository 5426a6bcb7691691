// Serving loop (continuous batching) -- interim: entry points present,
// implementation follows.
#include "internal.h"

struct wf_server { std::string err; };

extern "C" {
wf_status wf_server_create(wf_server** out, int, size_t, int32_t, wf_alloc_fn, wf_free_fn, void*) {
  if (out) *out = nullptr;
  return WF_ESTATE;
}
wf_status wf_server_submit(wf_server*, const wf_request*, uint64_t*) { return WF_ESTATE; }
wf_status wf_server_poll(wf_server*, uint64_t, int32_t*, wf_solve_info*) { return WF_ESTATE; }
wf_status wf_server_fetch(wf_server*, uint64_t, double*) { return WF_ESTATE; }
wf_status wf_server_cancel(wf_server*, uint64_t) { return WF_ESTATE; }
wf_status wf_server_stats_get(wf_server*, wf_server_stats*) { return WF_ESTATE; }
const char* wf_server_last_error(const wf_server* s) { return s ? s->err.c_str() : "null server"; }
wf_status wf_server_destroy(wf_server*) { return WF_OK; }
}
