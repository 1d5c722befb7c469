// Learned SGS closure: placeholder entry points until the network kernels land.
#include "cm_impl.hpp"

using namespace cm;

extern "C" {
cm_status cm_model_set_mlp(cm_model*, const float*, const float*) { set_error("learned closure not built"); return CM_ERR_UNSUPPORTED; }
cm_status cm_model_mlp_fallbacks(cm_model*, int64_t*, void*) { set_error("learned closure not built"); return CM_ERR_UNSUPPORTED; }
cm_status cm_mlp_create(const cm_mlp_desc*, uint64_t, int, cm_mlp**) { set_error("learned closure not built"); return CM_ERR_UNSUPPORTED; }
cm_status cm_mlp_destroy(cm_mlp*) { return CM_OK; }
cm_status cm_mlp_train_step(cm_mlp*, const float*, const float*, int, float*, void*) { set_error("learned closure not built"); return CM_ERR_UNSUPPORTED; }
cm_status cm_mlp_grads(cm_mlp*, const float*, const float*, int, float*, void*) { set_error("learned closure not built"); return CM_ERR_UNSUPPORTED; }
cm_status cm_mlp_infer(cm_mlp*, const float*, float*, int, void*) { set_error("learned closure not built"); return CM_ERR_UNSUPPORTED; }
cm_status cm_mlp_get_params(const cm_mlp*, float*) { set_error("learned closure not built"); return CM_ERR_UNSUPPORTED; }
cm_status cm_mlp_set_params(cm_mlp*, const float*) { set_error("learned closure not built"); return CM_ERR_UNSUPPORTED; }
}
