// bk_mlp.hip - window-predicting MLP: model handle, training and inference kernels,
// and the learned evaluation form.
#include <hip/hip_runtime.h>
#include "../../include/besselk.h"
#include "bk_internal.hpp"

namespace bk {
int bk_besselk_learned(const double*, const double*, double*, int64_t, const bk_params* prm, double, double, hipStream_t)
{
    return prm->model ? BK_EINVAL : BK_ENOMODEL;
}
int bk_matern_learned(const bk_locs*, const bk_params* prm, int32_t, int32_t, void*, double, double, hipStream_t)
{
    return prm->model ? BK_EINVAL : BK_ENOMODEL;
}
}  // namespace bk

struct bk_model { int dummy; };
extern "C" {
int bk_model_create(bk_model** m) { if (!m) return BK_EINVAL; *m = new bk_model(); return BK_OK; }
void bk_model_destroy(bk_model* m) { delete m; }
int bk_model_load(bk_model*, const char*) { return BK_EIO; }
int bk_model_save(const bk_model*, const char*) { return BK_EIO; }
int bk_model_train(bk_model*, const double*, const double*, int64_t, const bk_train_cfg*, float*, hipStream_t) { return BK_EINVAL; }
int bk_model_set_margins(bk_model*, double, double, double, double) { return BK_EINVAL; }
int bk_model_get_params(const bk_model*, float*) { return BK_EINVAL; }
int bk_model_set_params(bk_model*, const float*) { return BK_EINVAL; }
int bk_model_get_norm(const bk_model*, double*) { return BK_EINVAL; }
int bk_model_set_norm(bk_model*, const double*) { return BK_EINVAL; }
int bk_model_get_box(const bk_model*, double*) { return BK_EINVAL; }
int bk_model_set_box(bk_model*, const double*) { return BK_EINVAL; }
int bk_mlp_infer(const bk_model*, const float*, float*, int64_t, hipStream_t) { return BK_EINVAL; }
int bk_mlp_grad(const float*, const float*, const float*, const float*, int64_t, float*, float*, void*, size_t, hipStream_t) { return BK_EINVAL; }
size_t bk_mlp_grad_scratch_bytes(int64_t) { return 0; }
int bk_adam_step(float*, const float*, float*, float*, int64_t, int32_t, float, float, float, float, hipStream_t) { return BK_EINVAL; }
size_t bk_workspace_bytes(int64_t n) { return n > 0 ? (size_t)n * 8 + 256 : 256; }
}
