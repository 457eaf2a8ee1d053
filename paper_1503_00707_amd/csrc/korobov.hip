// korobov.hip -- the Boltzmann collision integral on Korobov lattice nodes
// (section 3.2, eqs. 3-6) applied in place to the post-transport state:
//   B_i = sum_k W f_j            (eq. 4, collision frequency)
//   C_i = sum_k W f_l f_m        (eq. 5, inverse-collision integral)
//   I_i = -f_i P_i B_i + C_i     (eq. 6, conservative correction)
//   f'_i = f_i + (dt / Kn) I_i,  W = V_box |xi_j - xi_i| / p.
// The trial tables are the same for every cell.  A workgroup takes a tile
// of CELLS cells whose rows sit in LDS node-major ([node][cell]), so the
// gather of one node for all cells of the tile is one contiguous vector
// read; each thread owns NV / T velocity nodes and keeps their B and C for
// every cell of the tile in registers.  A table entry (read once per tile)
// carries the three node indices and n = |k_j - k_i|^2 in grid units, so
// W = w0 dv sqrt(n) is a lookup in a small LDS table.  The five coefficients
// of P solve the conservation system in the scaled basis (1, xi/v,
// |xi|^2/v^2), v = the grid's half width (the span of eq. 6's (1, xi,
// |xi|^2): the same P), assembled from FP64 workgroup sums.
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

template <typename F, int NH, int T, int CELLS, int WPE>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_korobov(KorArgs a) {
    constexpr int NV = 8 * NH * NH * NH, R = NV / T, NW = 3 * (2 * NH - 1) * (2 * NH - 1) + 1;
    static_assert(NV % T == 0 && T % 64 == 0, "whole nodes per thread, whole waves");
    // a node's row of the tile, padded by 16 bytes so that rows start on
    // 16 different bank groups (random rows are gathered every trial)
    constexpr int RS = CELLS + 16 / int(sizeof(F));
    __shared__ __align__(16) F fs[NV * RS];
    __shared__ double Wn[NW];
    __shared__ double red[(T / 64) * CELLS * 20];
    __shared__ double dco[CELLS][5];
    F *f = static_cast<F *>(a.f);
    const int64_t c0 = int64_t(blockIdx.x) * CELLS;
    const int nc = int(min(int64_t(CELLS), a.n_cells - c0));
    for (int c = 0; c < CELLS; ++c)
        for (int v = threadIdx.x; v < NV; v += T) fs[v * RS + c] = c < nc ? f[(c0 + c) * NV + v] : F(0);
    const double wd = a.w0 * a.g.dv[0];
    for (int q = threadIdx.x; q < NW; q += T) Wn[q] = wd * sqrt(double(q));
    __syncthreads();
    // eqs. 4 and 5: each table entry once per tile, applied to every cell of it
    double b[R][CELLS], cc[R][CELLS];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CELLS; ++c) b[r][c] = cc[r][c] = 0.0;
    const uint64_t *tab = a.table + threadIdx.x;
    for (int k = 0; k < a.p; ++k, tab += NV) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t e = tab[r * T];
            const int j = int(e & 0xFFFFu), l = int((e >> 16) & 0xFFFFu), m = int((e >> 32) & 0xFFFFu);
            const double W = Wn[int(e >> 48)];
            F fj[CELLS];
            __builtin_memcpy(fj, fs + j * RS, sizeof fj);
#pragma unroll
            for (int c = 0; c < CELLS; ++c) b[r][c] += W * double(fj[c]);
            if (l != 0xFFFF) {
                F fl[CELLS], fm[CELLS];
                __builtin_memcpy(fl, fs + l * RS, sizeof fl);
                __builtin_memcpy(fm, fs + m * RS, sizeof fm);
#pragma unroll
                for (int c = 0; c < CELLS; ++c) cc[r][c] += W * double(fl[c]) * double(fm[c]);
            }
        }
    }
    // eq. 6: per cell the 5x5 conservation system in the scaled basis
    const double iv = 1.0 / a.vmax;
    double psi[R][5];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double xi[3];
        node_velocity<NH>(int(threadIdx.x) + r * T, a.g, xi);
        psi[r][0] = 1.0;
        psi[r][1] = xi[0] * iv;
        psi[r][2] = xi[1] * iv;
        psi[r][3] = xi[2] * iv;
        psi[r][4] = (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]) * iv * iv;
    }
    // per cell 20 sums (15 of the symmetric matrix, 5 of the right side):
    // wave sums into LDS, then one barrier, the wave totals, and one thread
    // per cell solves its system
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < CELLS; ++c) {
        double s[20];
#pragma unroll
        for (int q = 0; q < 20; ++q) s[q] = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double fb = double(fs[(int(threadIdx.x) + r * T) * RS + c]) * b[r][c];
            const double rr = cc[r][c] - fb;
            int q = 0;
#pragma unroll
            for (int x = 0; x < 5; ++x)
#pragma unroll
                for (int y = x; y < 5; ++y) s[q++] += psi[r][x] * psi[r][y] * fb;
#pragma unroll
            for (int x = 0; x < 5; ++x) s[15 + x] += psi[r][x] * rr;
        }
#pragma unroll
        for (int q = 0; q < 20; ++q) {
            const double t = wave_sum(s[q]);
            if (lane == 0) red[(wid * CELLS + c) * 20 + q] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < CELLS && int(threadIdx.x) < nc) {
        const int c = threadIdx.x;
        double sm[20];
        for (int q = 0; q < 20; ++q) {
            double t = 0.0;
            for (int w = 0; w < T / 64; ++w) t += red[(w * CELLS + c) * 20 + q];
            sm[q] = t;
        }
        double A[5][5], rv[5], d[5] = {0, 0, 0, 0, 0};
        int q = 0;
        for (int x = 0; x < 5; ++x)
            for (int y = x; y < 5; ++y) A[x][y] = A[y][x] = sm[q++];
        for (int x = 0; x < 5; ++x) rv[x] = sm[15 + x];
        if (!solve5(A, rv, d)) *a.flag = 1;
        for (int x = 0; x < 5; ++x) dco[c][x] = d[x];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CELLS; ++c) {
        if (c >= nc) break;
        const double d0 = dco[c][0], d1 = dco[c][1], d2 = dco[c][2], d3 = dco[c][3], d4 = dco[c][4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = int(threadIdx.x) + r * T;
            const double P = 1.0 + d0 + (d1 * psi[r][1] + d2 * psi[r][2] + d3 * psi[r][3]) + d4 * psi[r][4];
            const double fv = double(fs[i * RS + c]);
            const double I = -fv * P * b[r][c] + cc[r][c];
            f[(c0 + c) * NV + i] = F(fv + a.dt_kn * I);
        }
    }
}

}  // namespace
}  // namespace impl

template <typename F>
static hipError_t korobov_dispatch(const KorArgs &a, hipStream_t st) {
#define DVM_KOR(NH, T, CELLS, W)                                                                    \
    case NH:                                                                                       \
        hipLaunchKernelGGL((impl::k_korobov<F, NH, T, CELLS, W>), dim3(unsigned((a.n_cells + CELLS - 1) / CELLS)), \
                           dim3(T), 0, st, a);                                                     \
        break;
    switch (a.g.nh) {
        DVM_KOR(2, 64, 8, 3)
        DVM_KOR(4, 512, 8, 4)
        DVM_KOR(6, 576, 4, 3)
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
