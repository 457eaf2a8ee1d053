// sensor.cpp -- host side of the breakdown sensor, the network's training
// and the kinetic/fluid hybrid step (kernels in sensor_impl.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "solver_impl.h"

using namespace dvm;

static_assert(DVM_NOALLOC_MAX_BATCH == kNoAllocMaxBatch, "static scratch limit");

namespace {

SensorArgsPub sensor_args(const dvm_solver *s) {
    return SensorArgsPub{s->mom, s->tables, s->n, s->m->h0, s->p.tau_mode, s->p.tau_or_kn};
}

uint8_t *hyb_mask(const dvm_solver *s) { return reinterpret_cast<uint8_t *>(s->ws + s->off_hyb); }
uint8_t *hyb_prev(const dvm_solver *s) { return hyb_mask(s) + align256(size_t(s->n)); }
uint8_t *hyb_rows(const dvm_solver *s) { return hyb_mask(s) + 2 * align256(size_t(s->n)); }
double *hyb_flux(const dvm_solver *s) {
    return reinterpret_cast<double *>(s->ws + s->off_hyb + 3 * align256(size_t(s->n)));
}
double *hyb_face(const dvm_solver *s) {
    return reinterpret_cast<double *>(reinterpret_cast<char *>(hyb_flux(s)) +
                                      align256(size_t(s->n) * kFluxRecord * 8));
}

int check_net(const dvm_mlp *net, int64_t n) {
    if (!net || !net->ws || !net->params) return fail(DVM_ERR_WORKSPACE, "network not bound");
    if (n < 1 || n > net->max_batch) return fail(DVM_ERR_ARG, "batch of %lld outside [1, %lld]", (long long)n,
                                                 (long long)net->max_batch);
    return DVM_OK;
}

}  // namespace

namespace dvm {
// every cell kinetic (fresh state): called when a solver's state is replaced
hipError_t solver_reset_hybrid(dvm_solver *s, hipStream_t st) {
    if (!s->hybrid || !s->ws) return hipSuccess;
    return hipMemsetAsync(hyb_prev(s), 1, size_t(s->n), st);
}
uint8_t *solver_hybrid_prev(const dvm_solver *s) { return s->hybrid && s->ws ? hyb_prev(s) : nullptr; }
hipError_t solver_fluid_moments(const dvm_solver *s, double *out, hipStream_t st) {
    if (!s->hybrid_fluid) return hipSuccess;
    return launch_fluid_moments(hyb_mask(s), s->mom, out, s->n, st);
}
}  // namespace dvm

extern "C" {

int dvm_features(dvm_solver *s, float *x, void *stream) {
    clear_error();
    if (!s || !x) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    hipError_t e = launch_features(sensor_args(s), x, S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "features");
}

int dvm_labels(dvm_solver *s, float *r, void *stream) {
    clear_error();
    if (!s || !r) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    const hipError_t e = launch_labels(s->fp64, s->f[s->cur], r, s->n, s->g, S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "labels");
}

int dvm_mlp_create(int64_t max_batch, dvm_mlp **out) {
    clear_error();
    if (!out || max_batch < 1) return fail(DVM_ERR_ARG, "max_batch must be >= 1");
    dvm_mlp *net = new (std::nothrow) dvm_mlp();
    if (!net) return fail(DVM_ERR_ARG, "out of host memory");
    net->max_batch = max_batch;
    size_t o = 0;
    net->off_m = o;     o += align256(kMlpWeights * sizeof(float));
    net->off_v = o;     o += align256(kMlpWeights * sizeof(float));
    net->off_grad = o;  o += align256(kMlpWeights * sizeof(float));
    net->off_loss = o;  o += 256;
    net->off_lpart = o; o += align256(size_t((max_batch + 255) / 256) * sizeof(double));
    net->off_rec = o;   o += align256(size_t(max_batch) * kMlpRecord * sizeof(float));
    net->ws_bytes = o;
    *out = net;
    return DVM_OK;
}

int dvm_mlp_workspace_bytes(const dvm_mlp *net, size_t *bytes) {
    clear_error();
    if (!net || !bytes) return fail(DVM_ERR_ARG, "null argument");
    *bytes = net->ws_bytes;
    return DVM_OK;
}

int dvm_mlp_bind(dvm_mlp *net, float *params, void *ws) {
    clear_error();
    if (!net || !params || !ws) return fail(DVM_ERR_ARG, "null argument");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(DVM_ERR_ARG, "workspace must be 256-byte aligned");
    net->params = params;
    net->ws = static_cast<char *>(ws);
    net->t = 0;
    return DVM_OK;
}

int dvm_mlp_set_normalization(dvm_mlp *net, const float *x, int64_t n, void *stream) {
    clear_error();
    if (!net || !net->params || !x || n < 1) return fail(DVM_ERR_ARG, "bad argument");
    hipError_t e = launch_norm_stats(x, n, net->params, S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "normalisation");
}

int dvm_mlp_forward(const dvm_mlp *net, const float *x, int64_t n, int32_t mode, float *z, void *stream) {
    clear_error();
    if (!net || !net->params || !x || !z || n < 1) return fail(DVM_ERR_ARG, "bad argument");
    if (mode != 0 && mode != 1) return fail(DVM_ERR_ARG, "mode must be 0 (FP32) or 1 (matrix cores)");
    hipError_t e = launch_mlp_forward(net->params, x, n, mode, z, S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "forward");
}

int dvm_mlp_gradient(dvm_mlp *net, const float *x, const float *y, int64_t n, float pos_weight, void *stream) {
    clear_error();
    int rc = check_net(net, n);
    if (rc) return rc;
    if (!x || !y || !(pos_weight > 0)) return fail(DVM_ERR_ARG, "bad argument");
    hipError_t e = launch_train(net->params, x, y, n, pos_weight, net->rec(), net->lpart(), net->grad(), net->loss(),
                                S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "gradient");
}

int dvm_mlp_gradient_noalloc(const float *params, const float *x, const float *y, int64_t n, float pos_weight,
                             float *grad, double *loss, void *stream) {
    clear_error();
    if (!params || !x || !y || !grad || !loss || !(pos_weight > 0)) return fail(DVM_ERR_ARG, "bad argument");
    if (n < 1 || n > kNoAllocMaxBatch)
        return fail(DVM_ERR_WORKSPACE, "batch of %lld samples outside [1, %lld], the static scratch's limit",
                    (long long)n, (long long)kNoAllocMaxBatch);
    hipError_t e = launch_train_noalloc(params, x, y, n, pos_weight, grad, loss, S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "gradient (static scratch)");
}

int dvm_mlp_adam(dvm_mlp *net, float lr, void *stream) {
    clear_error();
    if (!net || !net->ws) return fail(DVM_ERR_WORKSPACE, "network not bound");
    if (!(lr > 0)) return fail(DVM_ERR_ARG, "lr must be > 0");
    net->t++;
    const double c1 = 1.0 - std::pow(0.9, double(net->t)), c2 = 1.0 - std::pow(0.999, double(net->t));
    hipError_t e = launch_adam(net->params, net->m(), net->v(), net->grad(), lr, float(c1), float(c2), S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "adam");
}

int dvm_mlp_train_step(dvm_mlp *net, const float *x, const float *y, int64_t n, float lr, float pos_weight,
                       void *stream) {
    int rc = dvm_mlp_gradient(net, x, y, n, pos_weight, stream);
    return rc ? rc : dvm_mlp_adam(net, lr, stream);
}

int dvm_mlp_buffers(const dvm_mlp *net, const float **grads, const double **loss) {
    clear_error();
    if (!net || !net->ws) return fail(DVM_ERR_WORKSPACE, "network not bound");
    if (grads) *grads = net->grad();
    if (loss) *loss = net->loss();
    return DVM_OK;
}

void dvm_destroy_mlp(dvm_mlp *net) { delete net; }

int dvm_sensor(dvm_solver *s, const dvm_mlp *net, double kappa, uint8_t *mask, float *score, void *stream) {
    clear_error();
    if (!s || !mask) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    if (net && !net->params) return fail(DVM_ERR_WORKSPACE, "network not bound");
    hipError_t e = launch_sensor(sensor_args(s), net ? net->params : nullptr, kappa, mask, score, S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "sensor");
}

int dvm_hybrid_step(dvm_solver *s, const uint8_t *mask, int32_t n_steps, double dt, double cfl, void *stream) {
    clear_error();
    if (!s || !mask) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    if (!s->hybrid) return fail(DVM_ERR_UNSUPPORTED, "create the solver with params.hybrid = 1");
    if (s->muscl) return fail(DVM_ERR_UNSUPPORTED, "the hybrid step is first order");
    if (n_steps < 0) return fail(DVM_ERR_ARG, "n_steps < 0");
    if (!(dt > 0)) {
        int rc = dvm_dt(s, cfl, &dt);
        if (rc) return rc;
    }
    hipStream_t st = S(stream);
    hipError_t e = launch_mask_eff(mask, hyb_mask(s), s->tables, s->n, st);
    if (e != hipSuccess) return hip_fail(e, "hybrid mask");
    const HybArgsPub h{hyb_mask(s), hyb_prev(s), hyb_rows(s), hyb_flux(s), hyb_face(s),
                       s->p.fluid_flux == DVM_FLUX_CLOSED ? 1 : 0, 0};
    for (int it = 0; it < n_steps; ++it) {
        StepArgs a = solver_step_args(s, dt);
        a.f_in = s->f[s->cur];
        a.f_out = s->f[s->cur ^ 1];
        e = launch_hybrid(s->fp64, a, h, st);
        if (e != hipSuccess) return hip_fail(e, "hybrid step");
        s->cur ^= 1;
        s->steps++;
        s->hybrid_fluid = true;  // conservative: the mask lives on the device
        if (s->p.check_every > 0 && s->steps % s->p.check_every == 0) {
            e = launch_global_sums(s->mom, s->tables, s->n, s->m->h0, s->partials(), kPartials, s->sums(), st);
            if (e != hipSuccess) return hip_fail(e, "global sums");
        }
    }
    return DVM_OK;
}

}  // extern "C"
