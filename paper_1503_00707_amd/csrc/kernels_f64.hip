// kernels_f64.hip -- step, init, moment and wall kernels for double storage.
#include "step_impl.h"

namespace dvm {

hipError_t launch_step_f64(const StepArgs &a, const StepConfig &cfg, hipStream_t st) {
    return impl::step_dispatch<double>(a, cfg, st);
}
hipError_t launch_step_batch_f64(const StepArgs *inst, const uint32_t *wg_end, int n_inst, uint32_t total_wg,
                                 int nh, const StepConfig &cfg, hipStream_t st) {
    return impl::step_batch_dispatch<double>(inst, wg_end, n_inst, total_wg, nh, cfg, st);
}
hipError_t launch_init_f64(const InitArgs &a, hipStream_t st) { return impl::init_dispatch<double>(a, st); }
hipError_t launch_moments_f64(const void *f, double *out, int64_t n, const VelGrid &g, hipStream_t st) {
    return impl::moments_dispatch<double>(f, out, n, g, st);
}
hipError_t launch_wall_den_f64(const void *m1, double *den, const VelGrid &g, hipStream_t st) {
    return impl::wall_den_dispatch<double>(m1, den, g, st);
}

}  // namespace dvm
