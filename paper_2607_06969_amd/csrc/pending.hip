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
}
