// pending.hip -- entry points not implemented yet (return NEPMI_UNSUPPORTED).
#include "model.hpp"
using namespace nepmi;
extern "C" {
int nepmi_backward_params(nepmi_model*, int32_t, const int64_t*, const double*, const float*, const int32_t*,
                          const double*, const float*, const double*, float*, void*) {
  set_error("not implemented");
  return NEPMI_UNSUPPORTED;
}
int nepmi_loss_grad(nepmi_model*, int32_t, const int64_t*, const double*, const float*, const int32_t*,
                    const double*, const float*, const double*, const double*, int32_t, double*, float*, void*) {
  set_error("not implemented");
  return NEPMI_UNSUPPORTED;
}
int nepmi_md_create(nepmi_model*, int32_t, const int64_t*, const double*, const float*, const float*,
                    const int32_t*, const double*, double, double, nepmi_md**, void*) {
  set_error("not implemented");
  return NEPMI_UNSUPPORTED;
}
int nepmi_md_step(nepmi_md*, int32_t, void*) { return NEPMI_UNSUPPORTED; }
int nepmi_md_get(nepmi_md*, float*, float*, float*, double*, double*, double*, void*) { return NEPMI_UNSUPPORTED; }
int nepmi_md_stats(nepmi_md*, int64_t*, int64_t*) { return NEPMI_UNSUPPORTED; }
void nepmi_md_destroy(nepmi_md*) {}
int nepmi_md_time_kernels(nepmi_md*, int32_t, double*, void*) { return NEPMI_UNSUPPORTED; }
}
