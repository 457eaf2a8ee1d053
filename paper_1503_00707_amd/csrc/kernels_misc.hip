// kernels_misc.hip -- global conservation sums, layout conversion, and the
// precision dispatch of the launch interface.
#include <hip/hip_runtime.h>

#include "step_impl.h"

namespace dvm {
namespace {

// Global sums sum_c V_c mom[k][c]: fixed chunks, then one block over the partials.
__global__ __launch_bounds__(256) void k_sums_stage1(const double *mom, const DevCell *cells, int64_t n, double h0,
                                                     double *partials) {
    __shared__ double red[4 * 5];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t c = lo + threadIdx.x; c < hi; c += 256) {
        const double h = h0 / double(1 << cells[c].level);
        const double V = h * h * h;
        for (int k = 0; k < 5; ++k) v[k] += V * mom[k * n + c];
    }
    impl::block_sum<256, 5>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) partials[blockIdx.x * 5 + k] = v[k];
}

__global__ __launch_bounds__(256) void k_sums_stage2(const double *partials, int n_part, double *out) {
    __shared__ double red[4 * 5];
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < n_part; b += 256)
        for (int k = 0; k < 5; ++k) v[k] += partials[b * 5 + k];
    impl::block_sum<256, 5>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) out[k] = v[k];
}

// The same two-level sums for many instances in two launches: workgroup
// (instance i, block p) of stage 1 covers the same cell range as block p of
// k_sums_stage1 for that instance, so both paths agree bitwise.
__global__ __launch_bounds__(256) void k_sums_batch1(const SumArgs *inst, int n_part) {
    __shared__ double red[4 * 5];
    const int i = blockIdx.x / n_part, blk = blockIdx.x % n_part;
    const SumArgs a = inst[i];
    const int64_t n = a.n;
    const int64_t chunk = (n + n_part - 1) / n_part;
    const int64_t lo = blk * chunk, hi = min(n, lo + chunk);
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t c = lo + threadIdx.x; c < hi; c += 256) {
        const double h = a.h0 / double(1 << a.cells[c].level);
        const double V = h * h * h;
        for (int k = 0; k < 5; ++k) v[k] += V * a.mom[k * n + c];
    }
    impl::block_sum<256, 5>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) a.partials[blk * 5 + k] = v[k];
}

__global__ __launch_bounds__(256) void k_sums_batch2(const SumArgs *inst, int n_part) {
    __shared__ double red[4 * 5];
    const SumArgs a = inst[blockIdx.x];
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < n_part; b += 256)
        for (int k = 0; k < 5; ++k) v[k] += a.partials[b * 5 + k];
    impl::block_sum<256, 5>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) a.out[k] = v[k];
}

// canonical index (kx*N + ky)*N + kz  <->  internal octant-major index
template <typename F>
__global__ __launch_bounds__(256) void k_canon(const F *src, F *dst, int nh, int to_canon) {
    const int64_t B = int64_t(nh) * nh * nh, NV = 8 * B, N = 2 * nh;
    const int64_t c = blockIdx.x;
    for (int64_t v = threadIdx.x; v < NV; v += 256) {
        const int64_t o = v / B, s = v % B;
        const int64_t ax = s / (nh * nh), ay = (s / nh) % nh, az = s % nh;
        const int64_t kx = (o >> 2) ? nh + ax : nh - 1 - ax;
        const int64_t ky = ((o >> 1) & 1) ? nh + ay : nh - 1 - ay;
        const int64_t kz = (o & 1) ? nh + az : nh - 1 - az;
        const int64_t vc = (kx * N + ky) * N + kz;
        if (to_canon) dst[c * NV + vc] = src[c * NV + v];
        else dst[c * NV + v] = src[c * NV + vc];
    }
}

}  // namespace

bool have_kernel(int nh, int threads, int wpe) { return impl::step_config_exists(nh, threads, wpe); }
bool have_regular_kernel(int nh, int threads, int wpe) { return impl::reg_config_exists(nh, threads, wpe); }
int list_kernels(int nh, int *threads, int *wpe, int cap) { return impl::step_config_list(nh, threads, wpe, cap); }

int default_threads(bool fp64, int nh) {
    switch (nh) {
    case 2: return 64;
    case 4: return 64;
    case 6: return 256;
    case 8: return 256;
    case 12: return 576;
    default: return 0;
    }
}

hipError_t launch_step(bool fp64, const StepArgs &a, const StepConfig &cfg, hipStream_t st) {
    return fp64 ? launch_step_f64(a, cfg, st) : launch_step_f32(a, cfg, st);
}

hipError_t launch_step_batch(bool fp64, const StepArgs *inst, const uint32_t *wg_end, int n_inst, uint32_t total_wg,
                             int nh, const StepConfig &cfg, hipStream_t st) {
    return fp64 ? launch_step_batch_f64(inst, wg_end, n_inst, total_wg, nh, cfg, st)
                : launch_step_batch_f32(inst, wg_end, n_inst, total_wg, nh, cfg, st);
}

hipError_t launch_global_sums_batch(const SumArgs *inst, int n_inst, int n_part, hipStream_t st) {
    hipLaunchKernelGGL(k_sums_batch1, dim3(unsigned(n_inst * n_part)), dim3(256), 0, st, inst, n_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sums_batch2, dim3(unsigned(n_inst)), dim3(256), 0, st, inst, n_part);
    return hipGetLastError();
}

hipError_t launch_init(bool fp64, const InitArgs &a, hipStream_t st) {
    return fp64 ? launch_init_f64(a, st) : launch_init_f32(a, st);
}

hipError_t launch_moments(bool fp64, const void *f, double *out, int64_t n, const VelGrid &g, hipStream_t st) {
    return fp64 ? launch_moments_f64(f, out, n, g, st) : launch_moments_f32(f, out, n, g, st);
}

hipError_t launch_wall_den(bool fp64, const void *m1, double *den, const VelGrid &g, hipStream_t st) {
    return fp64 ? launch_wall_den_f64(m1, den, g, st) : launch_wall_den_f32(m1, den, g, st);
}


hipError_t launch_global_sums(const double *mom, const DevCell *cells, int64_t n, double h0, double *partials,
                              int n_part, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_sums_stage1, dim3(unsigned(n_part)), dim3(256), 0, st, mom, cells, n, h0, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sums_stage2, dim3(1), dim3(256), 0, st, partials, n_part, out);
    return hipGetLastError();
}

hipError_t launch_to_canonical(bool fp64, bool to_canon, const void *src, void *dst, int64_t n, int nh,
                               hipStream_t st) {
    if (fp64)
        hipLaunchKernelGGL(k_canon<double>, dim3(unsigned(n)), dim3(256), 0, st, static_cast<const double *>(src),
                           static_cast<double *>(dst), nh, int(to_canon));
    else
        hipLaunchKernelGGL(k_canon<float>, dim3(unsigned(n)), dim3(256), 0, st, static_cast<const float *>(src),
                           static_cast<float *>(dst), nh, int(to_canon));
    return hipGetLastError();
}

}  // namespace dvm
