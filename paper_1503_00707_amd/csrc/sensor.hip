// sensor.hip -- launchers of the sensor, training and hybrid-step kernels
// (sensor_impl.h), both storage precisions.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sensor_impl.h"

namespace dvm {

// Static scratch of dvm_mlp_gradient_noalloc: the per-sample records and the
// per-block loss partials of up to kNoAllocMaxBatch samples.  Each GPU holds
// its own copy until the process ends; every call on a GPU shares it.
namespace {
constexpr size_t kScratchRec = (size_t(kNoAllocMaxBatch) * kMlpRecord * sizeof(float) + 255) & ~size_t(255);
constexpr size_t kScratchPart = (size_t((kNoAllocMaxBatch + 255) / 256) * sizeof(double) + 255) & ~size_t(255);
constexpr int kMaxDevices = 64;
constexpr int64_t kSensorSmallMesh = 65536;
}  // namespace
static __device__ __align__(256) char scratch[kScratchRec + kScratchPart];

// Device address of this GPU's scratch (the host-side name of the array is
// not a device address): looked up once per device, with it current.
static hipError_t scratch_on_device(char **out) {
    static std::mutex mu;
    static char *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<char *>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

static_assert(sizeof(SensorArgsPub) == sizeof(impl::FeatArgs), "argument layout");
static_assert(sizeof(HybArgsPub) == sizeof(impl::HybArgs), "argument layout");
static_assert(kMlpParams == impl::kParams && kMlpWeights == impl::kWeights, "parameter block");
static_assert(kMlpRecord == impl::kRec && kFluxRecord == impl::kFluxRec, "scratch records");
static_assert(kFaceRecord == 6 * 5, "face flux records");

static impl::FeatArgs feat(const SensorArgsPub &a) {
    impl::FeatArgs f;
    __builtin_memcpy(&f, &a, sizeof f);
    return f;
}

hipError_t launch_features(const SensorArgsPub &a, float *x, hipStream_t st) {
    hipLaunchKernelGGL(impl::k_features, dim3(unsigned((a.n + 255) / 256)), dim3(256), 0, st, feat(a), x);
    return hipGetLastError();
}

hipError_t launch_labels(bool fp64, const void *f, float *r, int64_t n, const VelGrid &g, hipStream_t st) {
    return fp64 ? impl::labels_dispatch<double>(f, r, n, g, st) : impl::labels_dispatch<float>(f, r, n, g, st);
}

hipError_t launch_mlp_forward(const float *params, const float *x, int64_t n, int mode, float *z, hipStream_t st) {
    if (mode == 0)
        hipLaunchKernelGGL(impl::k_mlp_fwd32, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, params, x, n, z);
    else
        hipLaunchKernelGGL(impl::k_mlp_fwd_mfma, dim3(unsigned((n + 63) / 64)), dim3(256), 0, st, params, x, n, z);
    return hipGetLastError();
}

hipError_t launch_sensor(const SensorArgsPub &a, const float *params, double kappa, uint8_t *mask, float *score,
                         hipStream_t st) {
    // below 1024 workgroups of 64 cells, one-wave workgroups of 16 cells
    if (a.n <= kSensorSmallMesh)
        hipLaunchKernelGGL(impl::k_sensor<16>, dim3(unsigned((a.n + 15) / 16)), dim3(64), 0, st, feat(a), params,
                           kappa, mask, score);
    else
        hipLaunchKernelGGL(impl::k_sensor<64>, dim3(unsigned((a.n + 63) / 64)), dim3(256), 0, st, feat(a), params,
                           kappa, mask, score);
    return hipGetLastError();
}

hipError_t launch_train(const float *params, const float *x, const float *y, int64_t n, float pos_weight,
                        float *rec, double *loss_part, float *grad, double *loss, hipStream_t st) {
    const unsigned nb = unsigned((n + 255) / 256);
    hipLaunchKernelGGL(impl::k_train_fb, dim3(nb), dim3(256), 0, st, params, x, y, n, pos_weight, rec, loss_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(impl::k_train_grads, dim3(unsigned((impl::kWeights + 255) / 256)), dim3(256), 0, st, rec, n,
                       loss_part, int(nb), grad, loss);
    return hipGetLastError();
}

hipError_t launch_train_noalloc(const float *params, const float *x, const float *y, int64_t n, float pos_weight,
                                float *grad, double *loss, hipStream_t st) {
    if (n < 1 || n > kNoAllocMaxBatch) return hipErrorInvalidValue;
    char *base = nullptr;
    hipError_t e = scratch_on_device(&base);
    if (e != hipSuccess) return e;
    // every record and partial the gradient kernel reads is written first by
    // the forward/backward kernel of the same call: nothing to clear
    return launch_train(params, x, y, n, pos_weight, reinterpret_cast<float *>(base),
                        reinterpret_cast<double *>(base + kScratchRec), grad, loss, st);
}

hipError_t launch_adam(float *params, float *m, float *v, const float *grad, float lr, float c1, float c2,
                       hipStream_t st) {
    hipLaunchKernelGGL(impl::k_adam, dim3(unsigned((impl::kWeights + 255) / 256)), dim3(256), 0, st, params, m, v,
                       grad, lr, c1, c2);
    return hipGetLastError();
}

hipError_t launch_norm_stats(const float *x, int64_t n, float *params, hipStream_t st) {
    hipLaunchKernelGGL(impl::k_norm_stats, dim3(impl::kIn), dim3(256), 0, st, x, n, params);
    return hipGetLastError();
}

hipError_t launch_mask_eff(const uint8_t *in, uint8_t *out, const DevCell *cells, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(impl::k_mask_eff, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, in, out, cells, n);
    return hipGetLastError();
}

hipError_t launch_fluid_moments(const uint8_t *mask, const double *mom, double *out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(impl::k_fluid_moments, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, mask, mom, out, n);
    return hipGetLastError();
}

hipError_t launch_hybrid(bool fp64, const StepArgs &a, const HybArgsPub &h, hipStream_t st) {
    impl::HybArgs hh;
    __builtin_memcpy(&hh, &h, sizeof hh);
    return fp64 ? impl::hybrid_dispatch<double>(a, hh, st) : impl::hybrid_dispatch<float>(a, hh, st);
}

}  // namespace dvm
