// Entry points declared in open.h whose kernels are not in this build yet.
#include "common.h"

extern "C" {
#define OPEN_STUB(ret, name, ...)                                     \
  ret name(__VA_ARGS__) { return OPEN_E_UNSUPPORTED; }
OPEN_STUB(open_status, open_predict, open_ctx *, const float *, int64_t, const float *, int32_t, int32_t, float *, const float *, const float *, int32_t, float, int32_t *, float *, int32_t *)
OPEN_STUB(open_status, open_mlp_create, open_ctx *, open_mlp **, int32_t, int32_t, int32_t, const float *)
OPEN_STUB(open_status, open_mlp_destroy, open_mlp *)
OPEN_STUB(open_status, open_mlp_get_weights, open_mlp *, float *)
OPEN_STUB(open_status, open_mlp_set_weights, open_mlp *, const float *)
OPEN_STUB(open_status, open_mlp_forward, open_mlp *, int64_t, const int64_t *, const int32_t *, const float *, float *)
OPEN_STUB(open_status, open_mlp_loss_grad, open_mlp *, int64_t, const int64_t *, const int32_t *, const float *, const float *, double *, float *)
OPEN_STUB(open_status, open_mlp_train_step, open_mlp *, int64_t, const int64_t *, const int32_t *, const float *, const float *, const int64_t *, int32_t, float, float *)
OPEN_STUB(open_status, open_mlp_foldin, open_mlp *, const float *, int64_t, const int64_t *, const int32_t *, const float *, float, float, int32_t, float *, uint8_t *, float *, int64_t *)
int64_t open_mlp_num_params(int32_t n, int32_t k, int32_t hidden) {
  return (int64_t)hidden * 2 * n + hidden + (int64_t)hidden * hidden + hidden + (int64_t)k * hidden + k;
}
}
