// Entry points declared in dbpeq.h that are not implemented yet.
#include "eq_common.h"

extern "C" {

size_t eq_backward_workspace_size(const eq_problem *) { return 0; }

eq_status eq_pd_backward(const eq_problem *, const eq_c32 *, const eq_c32 *, const eq_c32 *,
                         const float *, eq_c32 *, eq_c32 *, float *, void *, size_t, void *) {
  return EQ_ENOTSUP;
}

eq_status eq_fd_backward(const eq_problem *, const eq_c32 *, const eq_c32 *, const float *,
                         const eq_c32 *, const float *, eq_c32 *, eq_c32 *, float *, float *,
                         void *, size_t, void *) {
  return EQ_ENOTSUP;
}

eq_status eq_plan_create(eq_plan **out, const eq_sys *, int32_t, const int32_t *, int32_t, int32_t,
                         int32_t, float, const char *) {
  if (out) *out = nullptr;
  return EQ_ENOTSUP;
}

eq_status eq_plan_execute(eq_plan *, const eq_c32 *, const eq_c32 *, eq_c32 *, float *, int32_t *,
                          void *) {
  return EQ_ENOTSUP;
}

eq_status eq_plan_describe(const eq_plan *, int32_t *, int32_t *) { return EQ_ENOTSUP; }

eq_status eq_plan_destroy(eq_plan *) { return EQ_OK; }

}  // extern "C"
