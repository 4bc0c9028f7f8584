// Host-only stand-ins for the library's device-side functions, so that the
// host C++ (tree building, argument validation, handle lifetime) can be built
// and run under AddressSanitizer / UndefinedBehaviorSanitizer with g++ and no
// HIP.  Every stand-in reports OCCK_EHIP: the sanitized driver only exercises
// paths that never reach the GPU.
#include "../../paper_1708_05353_amd/csrc/occk_internal.hpp"

namespace occk {

static int32_t no_gpu() {
  set_error("sanitizer build: no device code");
  return OCCK_EHIP;
}

void device_free(Tree*) {}
void jstate_free(Tree*) {}
void nstate_free(Tree*) {}
int32_t near_K(Tree*, const double*, int64_t, int32_t, double*, int64_t, int32_t, void*) { return no_gpu(); }
int32_t near_K_counts(Tree*, int64_t*, int64_t*) { return no_gpu(); }
int32_t far_J(Tree*, const double*, int64_t, double*, int64_t, int32_t, void*) { return no_gpu(); }
int32_t far_K(Tree*, const double*, int64_t, int32_t, int32_t, int32_t, int32_t, int32_t, const occk_far_opts*,
              double*, int64_t, void*) { return no_gpu(); }
int32_t far_K_noalloc(Tree*, const double*, int64_t, int32_t, int32_t, int32_t, int32_t, int32_t,
                      const occk_far_opts*, double*, int64_t, void*) { return no_gpu(); }
int32_t debug_mfma_probe(int, int, int, int, double*) { return no_gpu(); }
int32_t debug_buffer(Tree*, int, double*, int64_t*) { return no_gpu(); }
int32_t profile_read(Tree*, double*, int64_t*) { return no_gpu(); }
int32_t workspace_info(Tree*, int32_t* jblock, int64_t* bytes) {
  if (jblock) *jblock = -1;
  if (bytes) *bytes = 0;
  return OCCK_OK;
}
int32_t pair_screen_info(Tree*, int64_t* carried, int32_t* jblock, int32_t*, int32_t, int32_t* nband) {
  *carried = 0;
  *jblock = 0;
  *nband = 0;
  return OCCK_OK;
}
int32_t batch_create(int, Tree* const*, const int32_t*, int, int, void**) { return no_gpu(); }
int32_t batch_run(void*, const double* const*, const int64_t*, double* const*, const int64_t*, void*) {
  return no_gpu();
}
int32_t batch_tune(void*, const double* const*, const int64_t*, double* const*, const int64_t*, void*, int32_t*) {
  return no_gpu();
}
int32_t batch_free(void*) { return OCCK_OK; }
int32_t batch_stage_times(void*, double*, int32_t*, int, int32_t*) { return no_gpu(); }
int32_t batch_shape(const void*, int32_t*, int32_t*, int, int32_t*) { return no_gpu(); }
int32_t selector_create(int32_t, void**) { return no_gpu(); }
int32_t selector_free(void*) { return OCCK_OK; }
int32_t selector_weights(void*, float*, const float*) { return no_gpu(); }
void selector_set_rule(void*, float, float) {}
int32_t selector_train(void*, const float*, const float*, int32_t, int32_t, int32_t, float, int32_t, float*, void*) {
  return no_gpu();
}
int32_t selector_grad(void*, const float*, const float*, int32_t, float*, float*, void*) { return no_gpu(); }
int32_t selector_predict(void*, const float*, int32_t, int32_t, float*, int32_t*, void*) { return no_gpu(); }
int32_t selector_save(const void*, const char*) { return no_gpu(); }
int32_t selector_load(void*, const char*) { return no_gpu(); }
int32_t selector_collect(Tree*, const double*, int64_t, int32_t, int32_t, int32_t, int32_t, int32_t, float*, float*,
                         int32_t*, void*) { return no_gpu(); }
int32_t rank_stats(Tree*, int64_t*) { return no_gpu(); }
bool selector_live(const void*) { return false; }

}  // namespace occk
