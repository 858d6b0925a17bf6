// Batched form: several independent plans iterated together.
#include "gswmtp_internal.h"

extern "C" {

int gswmtp_batch_create(gswmtp_batch **out, gswmtp_plan *const *plans, int n_plans,
                        void *stream) {
  if (out) *out = nullptr;
  (void)plans;
  (void)n_plans;
  (void)stream;
  return GSWMTP_E_UNSUPPORTED;
}

int gswmtp_batch_iterate(gswmtp_batch *b, int n_iter) {
  (void)b;
  (void)n_iter;
  return GSWMTP_E_UNSUPPORTED;
}

int gswmtp_batch_sync(gswmtp_batch *b) {
  (void)b;
  return GSWMTP_E_UNSUPPORTED;
}

int gswmtp_batch_destroy(gswmtp_batch *b) {
  (void)b;
  return GSWMTP_OK;
}

}  // extern "C"
