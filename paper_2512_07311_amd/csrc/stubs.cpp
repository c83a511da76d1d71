// Temporary: entry points not built yet.
#include "common.h"
extern "C" {
rcs_status rcs_svd_jacobi(int32_t, int32_t, double*, double*, double*, void*) { return RCS_ERR_UNSUPPORTED; }
rcs_status rcs_two_site(int32_t, int32_t, int32_t, const double*, const double*, const double*, int32_t, double*, void*) { return RCS_ERR_UNSUPPORTED; }
rcs_status rcs_rsvd(int32_t, int32_t, const double*, int32_t, int32_t, uint64_t, uint64_t, double*, double*, void*) { return RCS_ERR_UNSUPPORTED; }
rcs_status rcs_spectrum_features(const double*, int32_t, int32_t, int32_t, int32_t, int32_t, float*, void*) { return RCS_ERR_UNSUPPORTED; }
rcs_status rcs_mlp_forward(const float*, const float*, int32_t, float*, void*) { return RCS_ERR_UNSUPPORTED; }
rcs_status rcs_mlp_backward(const float*, const float*, const float*, int32_t, float*, float*, void*) { return RCS_ERR_UNSUPPORTED; }
rcs_status rcs_mlp_adam(float*, const float*, float*, float*, int32_t, int32_t, float, float, float, float, void*) { return RCS_ERR_UNSUPPORTED; }
}
