// kernels_f32.hip -- step, init, moment and wall kernels for float storage.
#include "sweep_impl.h"

namespace dvm {

hipError_t launch_step_f32(const StepArgs &a, const StepConfig &cfg, hipStream_t st) {
    return impl::step_dispatch<float>(a, cfg, st);
}
hipError_t launch_step_batch_f32(const StepArgs *inst, const uint32_t *wg_end, int n_inst, uint32_t total_wg,
                                 int nh, const StepConfig &cfg, hipStream_t st) {
    return impl::step_batch_dispatch<float>(inst, wg_end, n_inst, total_wg, nh, cfg, st);
}
hipError_t launch_init_f32(const InitArgs &a, hipStream_t st) { return impl::init_dispatch<float>(a, st); }
hipError_t launch_face_f32(const StepArgs &a, hipStream_t st) { return impl::face_dispatch<float>(a, st); }
hipError_t launch_moments_f32(const void *f, double *out, int64_t n, const VelGrid &g, hipStream_t st) {
    return impl::moments_dispatch<float>(f, out, n, g, st);
}
hipError_t launch_wall_den_f32(const void *m1, double *den, const VelGrid &g, hipStream_t st) {
    return impl::wall_den_dispatch<float>(m1, den, g, st);
}

static_assert(sizeof(UnitArgsPub) == sizeof(impl::UnitArgs), "argument layout");
static_assert(sizeof(TableArgsPub) == sizeof(impl::TableArgs), "argument layout");

hipError_t launch_unit_moments_f32(const UnitArgsPub &a, hipStream_t st) {
    impl::UnitArgs u;
    __builtin_memcpy(&u, &a, sizeof u);
    return impl::unit_dispatch<float>(u, st);
}
hipError_t launch_sweep_f32(const UnitArgsPub &a, int wg_per_cu, int n_cu, bool nt, hipStream_t st) {
    impl::UnitArgs u;
    __builtin_memcpy(&u, &a, sizeof u);
    return impl::sweep_dispatch<float>(u, wg_per_cu, n_cu, nt, st);
}
hipError_t launch_tables_f32(const TableArgsPub &a, hipStream_t st) {
    impl::TableArgs t;
    __builtin_memcpy(&t, &a, sizeof t);
    return impl::tables_dispatch<float>(t, st);
}
hipError_t launch_identity_f32(void *tab, int64_t n, int nh, hipStream_t st) {
    return impl::identity_dispatch<float>(tab, n, nh, st);
}
hipError_t launch_canon_relaxed_f32(const void *fstar, const void *tab, void *dst, int64_t n, int nh, hipStream_t st) {
    return impl::canon_relaxed_dispatch<float>(fstar, tab, dst, n, nh, st);
}
hipError_t launch_materialize_f32(void *fstar, void *tab, int64_t n, int nh, hipStream_t st) {
    return impl::materialize_dispatch<float>(fstar, tab, n, nh, st);
}

}  // namespace dvm
