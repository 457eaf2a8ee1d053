// korobov.hip -- the Boltzmann collision integral on Korobov lattice nodes
// (section 3.2, eqs. 3-6) applied in place to the post-transport state:
//   B_i = sum_k W f_j            (eq. 4, collision frequency)
//   C_i = sum_k W f_l f_m        (eq. 5, inverse-collision integral)
//   I_i = -f_i P_i B_i + C_i     (eq. 6, conservative correction)
//   f'_i = f_i + (dt / Kn) I_i,  W = V_box |xi_j - xi_i| / p.
// The trial tables are the same for every cell.  A workgroup takes a tile
// of CELLS cells: their rows sit in LDS (gathers at the table's indices are
// LDS reads), each table entry is read once per tile and applied to all of
// its cells, and B, C stay in LDS for the correction.  The five coefficients
// of P solve the conservation system in the scaled basis
// (1, xi/v, |xi|^2/v^2), v = the grid's half width (the span of eq. 6's
// (1, xi, |xi|^2): the same P), assembled from FP64 workgroup sums.
// The paper's own kernel runs one thread block per velocity node over all
// cells, f stored velocity-major and transposed for the correction; here the
// tables stream through L2 once per tile and f is never transposed.
#include <hip/hip_runtime.h>

#include "step_impl.h"

namespace dvm {
namespace impl {
namespace {

template <int NH>
__device__ __forceinline__ void node_velocity(int v, const VelGrid &g, double xi[3]) {
    constexpr int B = NH * NH * NH;
    const int o = v / B, s = v % B;
    const int ax = s / (NH * NH), ay = (s / NH) % NH, az = s % NH;
    xi[0] = ((o >> 2) ? 1.0 : -1.0) * (ax + 0.5) * g.dv[0];
    xi[1] = (((o >> 1) & 1) ? 1.0 : -1.0) * (ay + 0.5) * g.dv[1];
    xi[2] = ((o & 1) ? 1.0 : -1.0) * (az + 0.5) * g.dv[2];
}

// Gauss elimination with partial pivoting of a 5x5 system (one thread)
__device__ inline bool solve5(double A[5][5], double r[5], double x[5]) {
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int q = c + 1; q < 5; ++q)
            if (fabs(A[q][c]) > fabs(A[piv][c])) piv = q;
        if (A[piv][c] == 0.0) return false;
        if (piv != c) {
            for (int k = 0; k < 5; ++k) {
                const double t = A[c][k];
                A[c][k] = A[piv][k];
                A[piv][k] = t;
            }
            const double t = r[c];
            r[c] = r[piv];
            r[piv] = t;
        }
        for (int q = c + 1; q < 5; ++q) {
            const double m = A[q][c] / A[c][c];
            for (int k = c; k < 5; ++k) A[q][k] -= m * A[c][k];
            r[q] -= m * r[c];
        }
    }
    for (int q = 4; q >= 0; --q) {
        double s = r[q];
        for (int k = q + 1; k < 5; ++k) s -= A[q][k] * x[k];
        x[q] = s / A[q][q];
    }
    return true;
}

template <typename F, int NH, int CELLS>
__global__ __launch_bounds__(256) void k_korobov(KorArgs a) {
    constexpr int NV = 8 * NH * NH * NH, T = 256;
    __shared__ F fs[CELLS][NV];
    __shared__ double Bs[CELLS][NV], Cs[CELLS][NV];
    __shared__ double red[(T / 64) * 20];
    __shared__ double dco[CELLS][5];
    F *f = static_cast<F *>(a.f);
    const int64_t c0 = int64_t(blockIdx.x) * CELLS;
    const int nc = int(min(int64_t(CELLS), a.n_cells - c0));
    for (int c = 0; c < nc; ++c)
        for (int v = threadIdx.x; v < NV; v += T) fs[c][v] = f[(c0 + c) * NV + v];
    __syncthreads();
    // eqs. 4 and 5: each table entry once per tile, applied to every cell of it
    for (int i = threadIdx.x; i < NV; i += T) {
        double xi[3];
        node_velocity<NH>(i, a.g, xi);
        double b[CELLS], cc[CELLS];
#pragma unroll
        for (int c = 0; c < CELLS; ++c) b[c] = cc[c] = 0.0;
        for (int k = 0; k < a.p; ++k) {
            const uint64_t e = a.table[int64_t(k) * NV + i];
            const int j = int(e & 0xFFFFu), l = int((e >> 16) & 0xFFFFu), m = int((e >> 32) & 0xFFFFu);
            double xs[3];
            node_velocity<NH>(j, a.g, xs);
            const double gx = xs[0] - xi[0], gy = xs[1] - xi[1], gz = xs[2] - xi[2];
            const double W = a.w0 * sqrt(gx * gx + gy * gy + gz * gz);
            if (l != 0xFFFF) {
#pragma unroll
                for (int c = 0; c < CELLS; ++c) {
                    b[c] += W * double(fs[c][j]);
                    cc[c] += W * double(fs[c][l]) * double(fs[c][m]);
                }
            } else {
#pragma unroll
                for (int c = 0; c < CELLS; ++c) b[c] += W * double(fs[c][j]);
            }
        }
#pragma unroll
        for (int c = 0; c < CELLS; ++c) {
            Bs[c][i] = b[c];
            Cs[c][i] = cc[c];
        }
    }
    __syncthreads();
    // eq. 6: per cell the 5x5 conservation system in the scaled basis
    const double iv = 1.0 / a.vmax;
    for (int c = 0; c < nc; ++c) {
        double s[20];
#pragma unroll
        for (int q = 0; q < 20; ++q) s[q] = 0.0;
        for (int i = threadIdx.x; i < NV; i += T) {
            double xi[3];
            node_velocity<NH>(i, a.g, xi);
            const double psi[5] = {1.0, xi[0] * iv, xi[1] * iv, xi[2] * iv,
                                   (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]) * iv * iv};
            const double fb = double(fs[c][i]) * Bs[c][i];
            const double rr = Cs[c][i] - fb;
            int q = 0;
#pragma unroll
            for (int x = 0; x < 5; ++x)
#pragma unroll
                for (int y = x; y < 5; ++y) s[q++] += psi[x] * psi[y] * fb;
#pragma unroll
            for (int x = 0; x < 5; ++x) s[15 + x] += psi[x] * rr;
        }
        block_sum<T, 20>(s, red);
        if (threadIdx.x == 0) {
            double A[5][5], r[5], d[5] = {0, 0, 0, 0, 0};
            int q = 0;
            for (int x = 0; x < 5; ++x)
                for (int y = x; y < 5; ++y) A[x][y] = A[y][x] = s[q++];
            for (int x = 0; x < 5; ++x) r[x] = s[15 + x];
            if (!solve5(A, r, d)) *a.flag = 1;
            for (int x = 0; x < 5; ++x) dco[c][x] = d[x];
        }
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
        const double d0 = dco[c][0], d1 = dco[c][1], d2 = dco[c][2], d3 = dco[c][3], d4 = dco[c][4];
        for (int i = threadIdx.x; i < NV; i += T) {
            double xi[3];
            node_velocity<NH>(i, a.g, xi);
            const double P = 1.0 + d0 + (d1 * xi[0] + d2 * xi[1] + d3 * xi[2]) * iv +
                             d4 * (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]) * iv * iv;
            const double fv = double(fs[c][i]);
            const double I = -fv * P * Bs[c][i] + Cs[c][i];
            f[(c0 + c) * NV + i] = F(fv + a.dt_kn * I);
        }
    }
}

}  // namespace
}  // namespace impl

template <typename F>
static hipError_t korobov_dispatch(const KorArgs &a, hipStream_t st) {
#define DVM_KOR(NH, CELLS)                                                                         \
    case NH:                                                                                       \
        hipLaunchKernelGGL((impl::k_korobov<F, NH, CELLS>), dim3(unsigned((a.n_cells + CELLS - 1) / CELLS)), \
                           dim3(256), 0, st, a);                                                   \
        break;
    switch (a.g.nh) {
        DVM_KOR(2, 16)
        DVM_KOR(4, 4)
        DVM_KOR(6, 1)
    default: return hipErrorInvalidValue;
    }
#undef DVM_KOR
    return hipGetLastError();
}

bool korobov_supported(int nh) { return nh == 2 || nh == 4 || nh == 6; }

hipError_t launch_korobov(bool fp64, const KorArgs &a, hipStream_t st) {
    return fp64 ? korobov_dispatch<double>(a, st) : korobov_dispatch<float>(a, st);
}

}  // namespace dvm
