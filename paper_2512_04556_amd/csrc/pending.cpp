// Entry points whose kernels are not built yet: they validate nothing and
// report DISK_UNSUPPORTED.
#include "internal.hpp"

extern "C" {
int64_t disk_net_param_count(void) { return 0; }
size_t disk_net_workspace_size(int32_t) { return 0; }
disk_status disk_init_predict(const float*, const uint16_t*, const float*, float*, int32_t, void*, size_t,
                              hipStream_t) {
    return DISK_UNSUPPORTED;
}
disk_status disk_net_train_step(float*, float*, float*, int32_t, float, const uint16_t*, const float*, int32_t,
                                float*, void*, size_t, hipStream_t) {
    return DISK_UNSUPPORTED;
}
disk_status disk_net_prepare_inputs(const disk_batch_meta*, const disk_target*, const float*, uint16_t*, float*,
                                    hipStream_t) {
    return DISK_UNSUPPORTED;
}
disk_status disk_net_scatter_theta(const disk_batch_meta*, const disk_target*, const float*, float*, hipStream_t) {
    return DISK_UNSUPPORTED;
}
}
