// lbm.hip -- the lattice Boltzmann subset (section 4): D3Q19 / D3Q27 on the
// same octree, finite-volume upwind transport of eq. (2) for each lattice
// vector, then BGK relaxation toward the second-order equilibrium
//   f_eq = w rho (1 + c.u / cs^2 + (c.u)^2 / (2 cs^4) - |u|^2 / (2 cs^2)),  cs^2 = 1/3.
// With 19 or 27 values per cell a whole cell fits in one thread's registers:
// one thread per cell, f stored population-major ([q][cell]) so that the
// lanes of a wave read 64 consecutive cells of one population (coalesced),
// and the upwind neighbours' values are gathers served mostly by L2 (cells
// in Morton order).  Algorithmic traffic: read f once, write f once,
// 2 Q sizeof(F) bytes per cell, plus the 32-byte cell record.
#include <hip/hip_runtime.h>

#include "step_impl.h"

namespace dvm {
namespace {

// lattice vectors in canonical 3^3 order (kx, ky, kz in 0..2, c = k - 1),
// the 8 corners left out for D3Q19
template <int Q>
struct Lattice {
    int c[Q][3];
    double w[Q];
    constexpr Lattice() : c(), w() {
        int q = 0;
        for (int kx = 0; kx < 3; ++kx)
            for (int ky = 0; ky < 3; ++ky)
                for (int kz = 0; kz < 3; ++kz) {
                    const int c2 = (kx - 1) * (kx - 1) + (ky - 1) * (ky - 1) + (kz - 1) * (kz - 1);
                    if (Q == 19 && c2 == 3) continue;
                    c[q][0] = kx - 1;
                    c[q][1] = ky - 1;
                    c[q][2] = kz - 1;
                    w[q] = Q == 27 ? (c2 == 0 ? 8.0 / 27 : c2 == 1 ? 2.0 / 27 : c2 == 2 ? 1.0 / 54 : 1.0 / 216)
                                   : (c2 == 0 ? 1.0 / 3 : c2 == 1 ? 1.0 / 18 : 1.0 / 36);
                    ++q;
                }
    }
};

template <int Q>
__device__ constexpr Lattice<Q> kLat{};

__device__ __forceinline__ int face_kind(uint32_t meta, int f) { return int((meta >> (3 * f)) & 7u); }

// BUF: the state fits 32-bit byte offsets, so every access is a raw buffer
// access (per-lane 32-bit cell offset, the population's base as a scalar
// offset) instead of a 64-bit address per lane
template <typename F, int Q, bool BUF>
__global__ __launch_bounds__(256) void k_lbm(LbmArgs a) {
    const int64_t c = int64_t(impl::remap_cell(blockIdx.x, gridDim.x, a.xcd_log2)) * 256 + threadIdx.x;
    if (c >= a.n) return;
    const F *fi = static_cast<const F *>(a.f_in);
    F *fo = static_cast<F *>(a.f_out);
    const uint32_t bytes = BUF ? uint32_t(uint64_t(Q) * uint64_t(a.n) * sizeof(F)) : 0u;
    const impl::Rsrc ri = impl::rsrc(fi, bytes), ro = impl::rsrc(fo, bytes);
    auto ld = [&](int q, int64_t idx) -> F {
        if constexpr (BUF)
            return impl::bld<F>(ri, uint32_t(idx) * uint32_t(sizeof(F)), uint32_t(q) * uint32_t(a.n) * uint32_t(sizeof(F)));
        else
            return fi[q * a.n + idx];
    };
    const LbmCell rec = a.cells[c];
    const double h = a.h0 / double(1u << (rec.meta >> 24));
    const F r = F(a.dt / h);
    const int64_t n = a.n;
    // finer-face tuples of this cell follow each other in face order
    int fine_at[6];
    {
        int k = rec.fine;
        for (int f = 0; f < 6; ++f) {
            fine_at[f] = k;
            if (face_kind(rec.meta, f) == DVM_FACE_FINER) k += 4;
        }
    }
    F fs[Q];
    double rho = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const F own = ld(q, c);
        F acc = F(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int cb = kLat<Q>.c[q][b];
            if (cb == 0) continue;
            const int f = cb > 0 ? 2 * b : 2 * b + 1;  // the upwind face
            const int kind = face_kind(rec.meta, f);
            F up;
            if (kind == DVM_FACE_SAME || kind == DVM_FACE_COARSER) {
                up = ld(q, rec.nb[f]);
            } else if (kind == DVM_FACE_FINER) {
                const int32_t *t = a.fine + fine_at[f];
                up = F(0.25) * ((ld(q, t[0]) + ld(q, t[1])) + (ld(q, t[2]) + ld(q, t[3])));
            } else {
                up = own;  // outflow: zero gradient
            }
            acc += own - up;
        }
        const F v = own - r * acc;
        fs[q] = v;
        rho += double(v);
        mx += double(kLat<Q>.c[q][0]) * double(v);
        my += double(kLat<Q>.c[q][1]) * double(v);
        mz += double(kLat<Q>.c[q][2]) * double(v);
    }
    if (!(rho > 0.0)) *a.flag = 1;
    const double ux = mx / rho, uy = my / rho, uz = mz / rho;
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double cu = kLat<Q>.c[q][0] * ux + kLat<Q>.c[q][1] * uy + kLat<Q>.c[q][2] * uz;
        const double feq = kLat<Q>.w[q] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        const double v = double(fs[q]);
        const double out = a.euler ? v + a.relax * (feq - v) : feq + (v - feq) * a.relax;
        if constexpr (BUF)
            impl::bst<F, 0>(ro, uint32_t(c) * uint32_t(sizeof(F)), uint32_t(q) * uint32_t(n) * uint32_t(sizeof(F)), F(out));
        else
            fo[q * n + c] = F(out);
    }
}

// moments (rho, rho u, E = sum |c|^2 f / 2) of every cell, and the cell's
// volume-weighted contribution summed per block (first stage of the global sums)
template <typename F, int Q>
__global__ __launch_bounds__(256) void k_lbm_moments(const F *f, const LbmCell *cells, int64_t n, double h0,
                                                     double *mom, double *partials) {
    __shared__ double red[4 * 5];
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double v[5] = {0, 0, 0, 0, 0};
    if (c < n) {
        double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double x = double(f[q * n + c]);
            const int cx = kLat<Q>.c[q][0], cy = kLat<Q>.c[q][1], cz = kLat<Q>.c[q][2];
            m[0] += x;
            m[1] += cx * x;
            m[2] += cy * x;
            m[3] += cz * x;
            m[4] += 0.5 * double(cx * cx + cy * cy + cz * cz) * x;
        }
        for (int k = 0; k < 5; ++k) mom[k * n + c] = m[k];
        const double h = h0 / double(1u << (cells[c].meta >> 24));
        for (int k = 0; k < 5; ++k) v[k] = h * h * h * m[k];
    }
    impl::block_sum<256, 5>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) partials[blockIdx.x * 5 + k] = v[k];
}

__global__ __launch_bounds__(256) void k_lbm_sums(const double *partials, int nb, double *out) {
    __shared__ double red[4 * 5];
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int k = 0; k < 5; ++k) v[k] += partials[b * 5 + k];
    impl::block_sum<256, 5>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) out[k] = v[k];
}

// f_eq of (rho, u) per cell: prim [4][n]
template <typename F, int Q>
__global__ __launch_bounds__(256) void k_lbm_init(const double *prim, F *f, int64_t n, int *flag) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= n) return;
    const double rho = prim[c], ux = prim[n + c], uy = prim[2 * n + c], uz = prim[3 * n + c];
    if (!(rho > 0.0)) *flag = 1;
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double cu = kLat<Q>.c[q][0] * ux + kLat<Q>.c[q][1] * uy + kLat<Q>.c[q][2] * uz;
        f[q * n + c] = F(kLat<Q>.w[q] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

// population-major [Q][n] <-> canonical [n][27] (corners zero for D3Q19)
template <typename F, int Q>
__global__ __launch_bounds__(256) void k_lbm_canon(const F *src, F *dst, int64_t n, int to_canon) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= n) return;
    if (to_canon)
        for (int k = 0; k < 27; ++k) dst[c * 27 + k] = F(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = (kLat<Q>.c[q][0] + 1) * 9 + (kLat<Q>.c[q][1] + 1) * 3 + (kLat<Q>.c[q][2] + 1);
        if (to_canon) dst[c * 27 + k] = src[q * n + c];
        else dst[q * n + c] = src[c * 27 + k];
    }
}

template <typename F, int Q>
hipError_t run(const char *what, const LbmArgs &a, const void *p0, void *p1, double *p2, double *p3, int64_t n,
               double h0, int flagmode, hipStream_t st) {
    const dim3 g{unsigned((n + 255) / 256), 1, 1}, blk{256, 1, 1};
    switch (what[0]) {
    case 's':
        if (uint64_t(Q) * uint64_t(n) * sizeof(F) < (uint64_t(1) << 32))
            hipLaunchKernelGGL((k_lbm<F, Q, true>), g, blk, 0, st, a);
        else
            hipLaunchKernelGGL((k_lbm<F, Q, false>), g, blk, 0, st, a);
        break;
    case 'm':
        hipLaunchKernelGGL((k_lbm_moments<F, Q>), g, blk, 0, st, static_cast<const F *>(p0), a.cells, n, h0, p2, p3);
        break;
    case 'i':
        hipLaunchKernelGGL((k_lbm_init<F, Q>), g, blk, 0, st, static_cast<const double *>(p0), static_cast<F *>(p1),
                           n, a.flag);
        break;
    default:
        hipLaunchKernelGGL((k_lbm_canon<F, Q>), g, blk, 0, st, static_cast<const F *>(p0), static_cast<F *>(p1), n,
                           flagmode);
        break;
    }
    return hipGetLastError();
}

template <int Q>
hipError_t run_prec(bool fp64, const char *what, const LbmArgs &a, const void *p0, void *p1, double *p2, double *p3,
                    int64_t n, double h0, int flagmode, hipStream_t st) {
    return fp64 ? run<double, Q>(what, a, p0, p1, p2, p3, n, h0, flagmode, st)
                : run<float, Q>(what, a, p0, p1, p2, p3, n, h0, flagmode, st);
}

hipError_t dispatch(int q, bool fp64, const char *what, const LbmArgs &a, const void *p0, void *p1, double *p2,
                    double *p3, int64_t n, double h0, int flagmode, hipStream_t st) {
    if (q == 19) return run_prec<19>(fp64, what, a, p0, p1, p2, p3, n, h0, flagmode, st);
    if (q == 27) return run_prec<27>(fp64, what, a, p0, p1, p2, p3, n, h0, flagmode, st);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_lbm_step(int q, bool fp64, const LbmArgs &a, hipStream_t st) {
    return dispatch(q, fp64, "step", a, nullptr, nullptr, nullptr, nullptr, a.n, a.h0, 0, st);
}

hipError_t launch_lbm_moments(int q, bool fp64, const void *f, const LbmCell *cells, int64_t n, double h0,
                              double *mom, double *partials, double *sums, hipStream_t st) {
    LbmArgs a{};
    a.cells = cells;
    hipError_t e = dispatch(q, fp64, "moments", a, f, nullptr, mom, partials, n, h0, 0, st);
    if (e != hipSuccess || !sums) return e;
    hipLaunchKernelGGL(k_lbm_sums, dim3(1), dim3(256), 0, st, partials, int((n + 255) / 256), sums);
    return hipGetLastError();
}

hipError_t launch_lbm_init(int q, bool fp64, const double *prim, void *f, int64_t n, int *flag, hipStream_t st) {
    LbmArgs a{};
    a.flag = flag;
    return dispatch(q, fp64, "init", a, prim, f, nullptr, nullptr, n, 0.0, 0, st);
}

hipError_t launch_lbm_canon(int q, bool fp64, const void *src, void *dst, int64_t n, bool to_canon, hipStream_t st) {
    LbmArgs a{};
    return dispatch(q, fp64, "canon", a, src, dst, nullptr, nullptr, n, 0.0, to_canon ? 1 : 0, st);
}

}  // namespace dvm
