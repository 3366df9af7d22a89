// Batched copy (placeholder until the persistent batch kernel lands).
#include "host.hpp"

using namespace lm;

extern "C" {
llama_status llama_batch_create(uint32_t, const llama_view* const*, llama_view* const*, const char*, llama_batch** out) {
  if (out) *out = nullptr;
  return fail(LLAMA_ERR_UNSUPPORTED, "batched copy not built yet");
}
llama_status llama_batch_launch(llama_batch*, void*) { return fail(LLAMA_ERR_UNSUPPORTED, "batched copy not built yet"); }
llama_status llama_batch_launch_per_view(llama_batch*, void*) { return fail(LLAMA_ERR_UNSUPPORTED, "batched copy not built yet"); }
llama_status llama_batch_get_info(const llama_batch*, llama_batch_info*) { return fail(LLAMA_ERR_UNSUPPORTED, "batched copy not built yet"); }
llama_status llama_batch_destroy(llama_batch*) { return LLAMA_OK; }
}
