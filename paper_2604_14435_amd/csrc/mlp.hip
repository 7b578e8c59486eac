// Warm-start MLP kernels (bfloat16 matrix cores, float32 accumulation).
#include "common.h"

extern "C" {
int64_t dvq_mlp_param_count(const dvq_mlp_shape* s) {
    if (!s) return 0;
    return (int64_t)s->hidden * s->d_in + s->hidden + (int64_t)s->hidden * s->hidden + s->hidden +
           (int64_t)s->d_out * s->hidden + s->d_out;
}
size_t dvq_mlp_workspace_bytes(const dvq_mlp_shape* s, int32_t batch) {
    (void)s; (void)batch;
    return 0;
}
dvq_status dvq_mlp_forward(const dvq_mlp_shape*, const float*, const float*, int32_t, float*, float*,
                           float*, dvq_stream) {
    return dvq::fail(DVQ_EUNSUPPORTED, "mlp not built");
}
dvq_status dvq_mlp_loss_grad(const float*, const float*, int64_t, float*, double*, dvq_stream) {
    return dvq::fail(DVQ_EUNSUPPORTED, "mlp not built");
}
dvq_status dvq_mlp_backward(const dvq_mlp_shape*, const float*, const float*, const float*,
                            const float*, const float*, int32_t, float*, void*, size_t, dvq_stream) {
    return dvq::fail(DVQ_EUNSUPPORTED, "mlp not built");
}
dvq_status dvq_adamw_step(float*, const float*, float*, float*, int64_t, int32_t, float, float, float,
                          float, float, dvq_stream) {
    return dvq::fail(DVQ_EUNSUPPORTED, "mlp not built");
}
}
