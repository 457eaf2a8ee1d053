// kernels_f32.hip -- step, init, moment and wall kernels for float storage.
#include "step_impl.h"

namespace dvm {

hipError_t launch_step_f32(const StepArgs &a, const StepConfig &cfg, hipStream_t st) {
    return impl::step_dispatch<float>(a, cfg, st);
}
hipError_t launch_step_batch_f32(const StepArgs *inst, const uint32_t *wg_end, int n_inst, uint32_t total_wg,
                                 int nh, const StepConfig &cfg, hipStream_t st) {
    return impl::step_batch_dispatch<float>(inst, wg_end, n_inst, total_wg, nh, cfg, st);
}
hipError_t launch_init_f32(const InitArgs &a, hipStream_t st) { return impl::init_dispatch<float>(a, st); }
hipError_t launch_moments_f32(const void *f, double *out, int64_t n, const VelGrid &g, hipStream_t st) {
    return impl::moments_dispatch<float>(f, out, n, g, st);
}
hipError_t launch_wall_den_f32(const void *m1, double *den, const VelGrid &g, hipStream_t st) {
    return impl::wall_den_dispatch<float>(m1, den, g, st);
}

}  // namespace dvm
