// Serving loop (continuous batching) -- placeholder until the loop lands.
#include "common.hpp"
#include "litho_internal.hpp"

extern "C" int litho_serve_create(litho_bank_t *const *, int, const litho_serve_cfg_t *, litho_server_t **out) {
  if (out) *out = nullptr;
  litho::set_error("litho_serve_create: not built yet");
  return LITHO_E_UNSUPPORTED;
}
extern "C" int litho_serve_submit(litho_server_t *, const litho_request_t *, uint64_t *) {
  litho::set_error("litho_serve_submit: not built yet");
  return LITHO_E_UNSUPPORTED;
}
extern "C" int litho_serve_poll(litho_server_t *, uint64_t, float *, float *, litho_result_info_t *, int64_t) {
  litho::set_error("litho_serve_poll: not built yet");
  return LITHO_E_UNSUPPORTED;
}
extern "C" void litho_serve_destroy(litho_server_t *) {}
