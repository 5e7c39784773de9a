// Entry points declared in aicdf.h whose kernels are not built yet.
#include "internal.hpp"

using namespace aicdf;

#define PENDING(name) return fail(AICDF_EINVAL, #name " is not available in this build")

extern "C" {
aicdf_status mlmc_level_cir(const aicdf_cir_params*, uint32_t, uint64_t, int32_t, const aicdf_surrogate*,
                            uint64_t, uint64_t, aicdf_level_sums*, double*, void*) { PENDING(mlmc_level_cir); }
aicdf_status aicdf_surrogate_create(double, double, double, uint64_t, aicdf_surrogate**) {
  PENDING(aicdf_surrogate_create);
}
void aicdf_surrogate_destroy(aicdf_surrogate*) {}
aicdf_status aicdf_surrogate_set_params(aicdf_surrogate*, const float*, size_t) { PENDING(set_params); }
aicdf_status aicdf_surrogate_get_params(const aicdf_surrogate*, float*, size_t) { PENDING(get_params); }
aicdf_status aicdf_surrogate_forward(const aicdf_surrogate*, size_t, const float*, const float*, float*, void*) {
  PENDING(aicdf_surrogate_forward);
}
aicdf_status aicdf_surrogate_loss_grad(const aicdf_surrogate*, size_t, const float*, const float*, const float*,
                                       double*, float*, void*) { PENDING(aicdf_surrogate_loss_grad); }
aicdf_status aicdf_surrogate_make_data(const aicdf_surrogate*, uint64_t, size_t, float*, float*, float*, void*) {
  PENDING(aicdf_surrogate_make_data);
}
aicdf_status aicdf_surrogate_train(aicdf_surrogate*, size_t, const float*, const float*, const float*, uint32_t,
                                   uint32_t, float, uint64_t, double*, void*) { PENDING(aicdf_surrogate_train); }
aicdf_status aicdf_surrogate_info(const aicdf_surrogate*, double*, double*, double*) { PENDING(info); }
aicdf_status aicdf_surrogate_save(const aicdf_surrogate*, const char*) { PENDING(save); }
aicdf_status aicdf_surrogate_load(const char*, aicdf_surrogate**) { PENDING(load); }
}
