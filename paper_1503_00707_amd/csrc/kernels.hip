// kernels.hip -- gfx950 kernels of the DVM-BGK step.
//
// Layout.  f is [cell][velocity] with the velocity index innermost; the 8
// velocity sign groups ("octants") are contiguous blocks of B = NH^3 nodes,
// (-,-,-) first and the z sign fastest (section 3.1, step 1); inside an
// octant, slot s = (ax*NH + ay)*NH + az has |xi_b| = (a_b + 1/2) dv_b.  A
// workgroup owns one cell: thread t handles slots t, t+T, ... in every octant,
// so (a) the |xi| of a thread's slots are the same in all 8 octants and only
// the signs change, (b) within one octant all lanes read the same upwind
// neighbour row, so the upwind choice is wavefront-uniform (one scalar branch
// per octant and axis) and 64 lanes read 256 contiguous bytes of that row.
//
// One step per cell, fused in one pass over HBM (read f once, write f once):
//   transport   eq. (2) in flux form: f* = f - dt/h sum_b |xi_b| (f - f_up,b),
//               f_up the upwind neighbour (SAME/COARSER), the mean of the four
//               finer neighbours (FINER: 4 sub-faces of area (h/2)^2), or a
//               ghost value (inflow Maxwellian, own value at an outflow face,
//               diffuse-wall re-emission);
//   moments     FP64 sums w sum (1, xi, |xi|^2/2) f*, lane partials -> wave
//               butterfly -> LDS (the O(log n) tree of section 3.2);
//   Maxwellian  separable: 3N exponentials per cell, the 5x5 Gram system of
//               eq. (6) built from 15 one-dimensional sums and solved in FP64;
//   relaxation  f' = e f* + (1-e) Mt, Mt = C g_x g_y g_z (P_x + P_y + P_z).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace dvm {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum K values over the workgroup; every thread receives the same totals
// (fixed combination order, so the result is deterministic).
template <int T, int K>
__device__ inline void block_sum(double (&v)[K], double *scratch) {
    constexpr int NW = (T + 63) / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) scratch[wid * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += scratch[w * K + k];
        v[k] = s;
    }
    __syncthreads();
}

// Workgroups are dispatched round-robin over the 8 XCDs; this gives each XCD
// runs of g consecutive cells (a bijection on [0, nb)).
__device__ inline int64_t remap_cell(int64_t b, int64_t nb, int g) {
    if (g <= 1) return b;
    const int64_t chunk = 8 * int64_t(g);
    const int64_t full = nb - nb % chunk;
    if (b >= full) return b;
    const int64_t xcd = b % 8, local = b / 8;
    return (local / g) * chunk + xcd * g + (local % g);
}

template <typename F, int NH>
struct MaxwellSmem {
    static constexpr int N = 2 * NH;
    double g[3][N];
    double c[3][N];
    double S[15];
    double d[5];
    double C;
    F tab[3][N][2];  // (G, P) per axis and node
};

// Corrected discrete Maxwellian of (rho, u, T) as separable tables:
//   Mt_i = C g_x g_y g_z (1 + d.phi_i),  phi = (1, cx, cy, cz, |c|^2),
//   c = (xi - u)/sqrt(T), g = exp(-c^2/2), C = rho (2 pi T)^(-3/2).
// d solves G d = r with G_ab = w sum_i phi_a phi_b M_i (eq. 6's five
// conservation equations in a centred basis that spans the same polynomials)
// and r = (rho, 0, 0, 0, 3 rho) - G[:,0], the phi-moments of the target minus
// those of the raw Maxwellian.  Every G entry is a product of 1D sums
// S_b,p = dv_b sum_k c_k^p g_k, so the cost is O(N), not O(N^3).
// tab[0] carries C * mfac so that the caller's M' = mfac * Mt.
template <typename F, int NH, int T>
__device__ void maxwell_tables(MaxwellSmem<F, NH> &sm, double rho, const double u[3], double Tt, double mfac,
                               const VelGrid &g) {
    constexpr int N = 2 * NH;
    const int tid = threadIdx.x;
    const double rsT = 1.0 / sqrt(Tt);
    for (int j = tid; j < 3 * N; j += T) {
        const int b = j / N, k = j % N;
        const double xi = (double(k - NH) + 0.5) * g.dv[b];
        const double cc = (xi - u[b]) * rsT;
        sm.g[b][k] = exp(-0.5 * cc * cc);
        sm.c[b][k] = cc;
    }
    __syncthreads();
    if (tid < 15) {
        const int b = tid / 5, p = tid % 5;
        double s = 0.0;
        for (int k = 0; k < N; ++k) {
            double t = sm.g[b][k];
            const double cc = sm.c[b][k];
            for (int q = 0; q < p; ++q) t *= cc;
            s += t;
        }
        sm.S[tid] = s * g.dv[b];
    }
    __syncthreads();
    if (tid == 0) {
        const double *X = &sm.S[0], *Y = &sm.S[5], *Z = &sm.S[10];
        double A[5][5], r[5];
        A[0][0] = X[0] * Y[0] * Z[0];
        A[0][1] = X[1] * Y[0] * Z[0];
        A[0][2] = X[0] * Y[1] * Z[0];
        A[0][3] = X[0] * Y[0] * Z[1];
        A[0][4] = X[2] * Y[0] * Z[0] + X[0] * Y[2] * Z[0] + X[0] * Y[0] * Z[2];
        A[1][1] = X[2] * Y[0] * Z[0];
        A[1][2] = X[1] * Y[1] * Z[0];
        A[1][3] = X[1] * Y[0] * Z[1];
        A[1][4] = X[3] * Y[0] * Z[0] + X[1] * Y[2] * Z[0] + X[1] * Y[0] * Z[2];
        A[2][2] = X[0] * Y[2] * Z[0];
        A[2][3] = X[0] * Y[1] * Z[1];
        A[2][4] = X[2] * Y[1] * Z[0] + X[0] * Y[3] * Z[0] + X[0] * Y[1] * Z[2];
        A[3][3] = X[0] * Y[0] * Z[2];
        A[3][4] = X[2] * Y[0] * Z[1] + X[0] * Y[2] * Z[1] + X[0] * Y[0] * Z[3];
        A[4][4] = X[4] * Y[0] * Z[0] + X[0] * Y[4] * Z[0] + X[0] * Y[0] * Z[4] +
                  2.0 * (X[2] * Y[2] * Z[0] + X[2] * Y[0] * Z[2] + X[0] * Y[2] * Z[2]);
        for (int i = 1; i < 5; ++i)
            for (int j = 0; j < i; ++j) A[i][j] = A[j][i];
        const double C = rho * pow(kTwoPi * Tt, -1.5);
        const double t0 = rho / C;
        r[0] = t0 - A[0][0];
        r[1] = -A[1][0];
        r[2] = -A[2][0];
        r[3] = -A[3][0];
        r[4] = 3.0 * t0 - A[4][0];
        // symmetric positive definite: elimination without pivoting
        for (int k = 0; k < 5; ++k)
            for (int i = k + 1; i < 5; ++i) {
                const double q = A[i][k] / A[k][k];
                for (int j = k; j < 5; ++j) A[i][j] -= q * A[k][j];
                r[i] -= q * r[k];
            }
        double d[5];
        for (int i = 4; i >= 0; --i) {
            double s = r[i];
            for (int j = i + 1; j < 5; ++j) s -= A[i][j] * d[j];
            d[i] = s / A[i][i];
        }
        for (int i = 0; i < 5; ++i) sm.d[i] = d[i];
        sm.C = C;
    }
    __syncthreads();
    for (int j = tid; j < 3 * N; j += T) {
        const int b = j / N, k = j % N;
        const double cc = sm.c[b][k];
        double P;
        if (b == 0) P = 1.0 + sm.d[0] + sm.d[1] * cc + sm.d[4] * cc * cc;
        else P = sm.d[1 + b] * cc + sm.d[4] * cc * cc;
        const double G = b == 0 ? sm.g[b][k] * sm.C * mfac : sm.g[b][k];
        sm.tab[b][k][0] = F(G);
        sm.tab[b][k][1] = F(P);
    }
    __syncthreads();
}

template <int NH>
__device__ inline void slot_axes(int s, int &ax, int &ay, int &az) {
    ax = s / (NH * NH);
    ay = (s / NH) % NH;
    az = s % NH;
}

// Write f' = e*fs + M' for the slots of this thread, M' from the tables.
template <typename F, int NH, int T, int S>
__device__ inline void relax_store(const MaxwellSmem<F, NH> &sm, const F (&fo)[8][S], F e, F *out) {
    constexpr int B = NH * NH * NH;
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int s = threadIdx.x + q * T;
        if (S * T > B && s >= B) continue;
        int a3[3];
        slot_axes<NH>(s, a3[0], a3[1], a3[2]);
        F G[3][2], P[3][2];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            G[b][0] = sm.tab[b][NH - 1 - a3[b]][0];
            G[b][1] = sm.tab[b][NH + a3[b]][0];
            P[b][0] = sm.tab[b][NH - 1 - a3[b]][1];
            P[b][1] = sm.tab[b][NH + a3[b]][1];
        }
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int ox = o >> 2, oy = (o >> 1) & 1, oz = o & 1;
            const F M = G[0][ox] * G[1][oy] * G[2][oz] * ((P[0][ox] + P[1][oy]) + P[2][oz]);
            out[o * B + s] = e * fo[o][q] + M;
        }
    }
}

template <typename F>
struct Upwind {
    const F *p[4];
    int n;       // 1 or 4 rows; 0: the cell's own value
    F scale;
};

// Source of the inflow through upwind face uf for the current octant.
template <typename F>
__device__ inline Upwind<F> upwind_source(const DevCell &cell, int uf, const F *fin, int64_t nv, const StepArgs &a,
                                          const double *rho_w) {
    Upwind<F> u;
    u.n = 1;
    u.scale = F(1);
    const int32_t *nb = cell.nbr[uf];
    switch (cell.type[uf]) {
    case DVM_FACE_SAME:
    case DVM_FACE_COARSER: u.p[0] = fin + int64_t(nb[0]) * nv; break;
    case DVM_FACE_FINER:
        u.n = 4;
        u.scale = F(0.25);
        for (int q = 0; q < 4; ++q) u.p[q] = fin + int64_t(nb[q]) * nv;
        break;
    case DVM_FACE_INFLOW: u.p[0] = static_cast<const F *>(a.ghost_in); break;
    case DVM_FACE_WALL:
        u.p[0] = static_cast<const F *>(a.wall_m1);
        u.scale = F(rho_w[uf]);
        break;
    default: u.n = 0; u.p[0] = nullptr; break;  // OUTFLOW: zero gradient
    }
    return u;
}

template <typename F>
__device__ inline F upwind_value(const Upwind<F> &u, int idx, F own) {
    if (u.n == 0) return own;
    if (u.n == 1) return u.scale * u.p[0][idx];
    return u.scale * ((u.p[0][idx] + u.p[1][idx]) + (u.p[2][idx] + u.p[3][idx]));
}

template <typename F, int NH, int T>
__global__ __launch_bounds__(T) void k_step(StepArgs a) {
    constexpr int B = NH * NH * NH;
    constexpr int64_t NV = 8 * B;
    constexpr int S = (B + T - 1) / T;
    constexpr int NW = (T + 63) / 64;
    __shared__ double red[NW * 5];
    __shared__ double rho_w[6];
    __shared__ MaxwellSmem<F, NH> sm;

    const int tid = threadIdx.x;
    const int64_t c = remap_cell(blockIdx.x, gridDim.x, a.xcd_group);
    const DevCell &cell = a.cells[c];
    const F *fin = static_cast<const F *>(a.f_in);
    const F *own = fin + c * NV;
    const double dth = a.dt / (a.h0 / double(1 << cell.level));

    // own values of every slot and octant, kept in registers for the step
    F fo[8][S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int s = tid + q * T;
        const bool ok = !(S * T > B) || s < B;
#pragma unroll
        for (int o = 0; o < 8; ++o) fo[o][q] = ok ? own[o * B + s] : F(0);
    }

    // diffuse walls: density of the re-emitted Maxwellian (zero net mass flux)
    if (cell.flags & 1) {
        for (int f = 0; f < 6; ++f) {
            if (cell.type[f] != DVM_FACE_WALL) continue;
            const int axis = f >> 1, side = f & 1;
            double v[1] = {0.0};
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int s = tid + q * T;
                if (S * T > B && s >= B) continue;
                int a3[3];
                slot_axes<NH>(s, a3[0], a3[1], a3[2]);
                const double xa = (a3[axis] + 0.5) * a.g.dv[axis];
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const int sb = axis == 0 ? (o >> 2) : axis == 1 ? ((o >> 1) & 1) : (o & 1);
                    if (sb == side) v[0] += xa * double(fo[o][q]);  // leaving through this face
                }
            }
            block_sum<T, 1>(v, red);
            if (tid == 0) rho_w[f] = v[0] / a.wall_den[f];
        }
        __syncthreads();
    }

    // transport and FP64 moment partials
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int s = tid + q * T;
        if (S * T > B && s >= B) continue;
        int a3[3];
        slot_axes<NH>(s, a3[0], a3[1], a3[2]);
        const double xa = (a3[0] + 0.5) * a.g.dv[0];
        const double ya = (a3[1] + 0.5) * a.g.dv[1];
        const double za = (a3[2] + 0.5) * a.g.dv[2];
        const F nux = F(dth * xa), nuy = F(dth * ya), nuz = F(dth * za);
        double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int ox = o >> 2, oy = (o >> 1) & 1, oz = o & 1;
            // a positive component enters through the low face, a negative one through the high face
            const Upwind<F> ux = upwind_source<F>(cell, 0 + (ox ? 0 : 1), fin, NV, a, rho_w);
            const Upwind<F> uy = upwind_source<F>(cell, 2 + (oy ? 0 : 1), fin, NV, a, rho_w);
            const Upwind<F> uz = upwind_source<F>(cell, 4 + (oz ? 0 : 1), fin, NV, a, rho_w);
            const int idx = o * B + s;
            const F v = fo[o][q];
            const F acc = nux * (v - upwind_value(ux, idx, v)) + nuy * (v - upwind_value(uy, idx, v)) +
                          nuz * (v - upwind_value(uz, idx, v));
            const F fs = v - acc;
            fo[o][q] = fs;
            const double d = double(fs);
            s0 += d;
            sx += ox ? d : -d;
            sy += oy ? d : -d;
            sz += oz ? d : -d;
        }
        m[0] += s0;
        m[1] += xa * sx;
        m[2] += ya * sy;
        m[3] += za * sz;
        m[4] += 0.5 * (xa * xa + ya * ya + za * za) * s0;
    }
    block_sum<T, 5>(m, red);

    const double w = a.g.w;
    const double rho = w * m[0];
    double u[3] = {w * m[1] / rho, w * m[2] / rho, w * m[3] / rho};
    const double E = w * m[4];
    const double Tt = (2.0 * E / rho - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / 3.0;
    const bool bad = !(rho > 0.0) || !(Tt > 0.0);
    if (tid == 0) {
        const int64_t n = a.n_cells;
        a.mom[c] = rho;
        a.mom[n + c] = w * m[1];
        a.mom[2 * n + c] = w * m[2];
        a.mom[3 * n + c] = w * m[3];
        a.mom[4 * n + c] = E;
        if (bad) *a.flag = 1;
    }
    F *out = static_cast<F *>(a.f_out) + c * NV;
    if (bad || a.collision == DVM_COLL_OFF) {
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int s = tid + q * T;
            if (S * T > B && s >= B) continue;
#pragma unroll
            for (int o = 0; o < 8; ++o) out[o * B + s] = fo[o][q];
        }
        return;
    }
    const double tau = a.tau_mode == DVM_TAU_HS ? a.tau_or_kn / (rho * sqrt(Tt)) : a.tau_or_kn;
    double e, mfac;
    if (a.collision == DVM_COLL_EULER) {
        e = 1.0 - a.dt / tau;
        mfac = a.dt / tau;
    } else {
        e = exp(-a.dt / tau);
        mfac = -expm1(-a.dt / tau);
    }
    maxwell_tables<F, NH, T>(sm, rho, u, Tt, mfac, a.g);
    relax_store<F, NH, T, S>(sm, fo, F(e), out);
}

// f := corrected Maxwellian of a prescribed state (init and ghost rows).
template <typename F, int NH, int T>
__global__ __launch_bounds__(T) void k_init(InitArgs a) {
    constexpr int B = NH * NH * NH;
    constexpr int64_t NV = 8 * B;
    constexpr int S = (B + T - 1) / T;
    __shared__ MaxwellSmem<F, NH> sm;
    const int64_t c = blockIdx.x;
    double p[5];
    for (int k = 0; k < 5; ++k) p[k] = a.prim ? a.prim[k * a.n + c] : a.prim0[k];
    const double rho = p[0], u[3] = {p[1], p[2], p[3]}, Tt = p[4];
    F *out = static_cast<F *>(a.f_out) + c * NV;
    if (!(rho > 0.0) || !(Tt > 0.0)) {
        if (threadIdx.x == 0) *a.flag = 1;
        return;
    }
    if (threadIdx.x == 0 && a.mom) {
        a.mom[c] = rho;
        for (int b = 0; b < 3; ++b) a.mom[(1 + b) * a.n + c] = rho * u[b];
        a.mom[4 * a.n + c] = 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + 1.5 * rho * Tt;
    }
    maxwell_tables<F, NH, T>(sm, rho, u, Tt, 1.0, a.g);
    F zero[8][S];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
        for (int o = 0; o < 8; ++o) zero[o][q] = F(0);
    relax_store<F, NH, T, S>(sm, zero, F(0), out);
}

// FP64 conserved moments of stored states.
template <typename F, int NH, int T>
__global__ __launch_bounds__(T) void k_moments(const F *f, double *out, int64_t n, VelGrid g) {
    constexpr int B = NH * NH * NH;
    constexpr int64_t NV = 8 * B;
    constexpr int NW = (T + 63) / 64;
    __shared__ double red[NW * 5];
    const int64_t c = blockIdx.x;
    const F *row = f + c * NV;
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = threadIdx.x; s < B; s += T) {
        int a3[3];
        slot_axes<NH>(s, a3[0], a3[1], a3[2]);
        const double xa = (a3[0] + 0.5) * g.dv[0], ya = (a3[1] + 0.5) * g.dv[1], za = (a3[2] + 0.5) * g.dv[2];
        double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        for (int o = 0; o < 8; ++o) {
            const double d = double(row[o * B + s]);
            s0 += d;
            sx += (o >> 2) ? d : -d;
            sy += ((o >> 1) & 1) ? d : -d;
            sz += (o & 1) ? d : -d;
        }
        m[0] += s0;
        m[1] += xa * sx;
        m[2] += ya * sy;
        m[3] += za * sz;
        m[4] += 0.5 * (xa * xa + ya * ya + za * za) * s0;
    }
    block_sum<T, 5>(m, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) out[k * n + c] = g.w * m[k];
}

// Wall denominators: sum over velocities entering the fluid through face f
// (xi.n < 0, n the outward normal of the fluid cell) of |xi.n| M1.
template <typename F, int NH>
__global__ __launch_bounds__(256) void k_wall_den(const F *m1, double *den, VelGrid g) {
    constexpr int B = NH * NH * NH;
    __shared__ double red[4 * 6];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int s = threadIdx.x; s < B; s += 256) {
        int a3[3];
        slot_axes<NH>(s, a3[0], a3[1], a3[2]);
        for (int o = 0; o < 8; ++o) {
            const int sg[3] = {o >> 2, (o >> 1) & 1, o & 1};
            const double val = double(m1[o * B + s]);
            for (int f = 0; f < 6; ++f) {
                const int axis = f >> 1, side = f & 1;
                if (sg[axis] != side) v[f] += (a3[axis] + 0.5) * g.dv[axis] * val;
            }
        }
    }
    block_sum<256, 6>(v, red);
    if (threadIdx.x == 0)
        for (int f = 0; f < 6; ++f) den[f] = v[f];
}

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
    block_sum<256, 5>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) partials[blockIdx.x * 5 + k] = v[k];
}

__global__ __launch_bounds__(256) void k_sums_stage2(const double *partials, int n_part, double *out) {
    __shared__ double red[4 * 5];
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < n_part; b += 256)
        for (int k = 0; k < 5; ++k) v[k] += partials[b * 5 + k];
    block_sum<256, 5>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) out[k] = v[k];
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

// ---------------------------------------------------------------------------
// instantiation tables
// ---------------------------------------------------------------------------

#define DVM_STEP_CONFIGS(X) \
    X(2, 64)                \
    X(4, 64)                \
    X(6, 64)                \
    X(6, 256)               \
    X(8, 256)               \
    X(8, 512)               \
    X(12, 192)              \
    X(12, 576)

template <typename F>
hipError_t step_dispatch(int nh, int threads, const StepArgs &a, hipStream_t st) {
#define X(NH, T)                                                                      \
    if (nh == NH && threads == T) {                                                   \
        hipLaunchKernelGGL((k_step<F, NH, T>), dim3(unsigned(a.n_cells)), dim3(T), 0, st, a); \
        return hipGetLastError();                                                     \
    }
    DVM_STEP_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

template <typename F>
int default_threads_t(int nh) {
    switch (nh) {
    case 2: return 64;
    case 4: return 64;
    case 6: return 256;
    case 8: return 256;
    case 12: return sizeof(F) == 8 ? 576 : 192;
    default: return 0;
    }
}

template <typename F>
hipError_t init_dispatch(const InitArgs &a, hipStream_t st) {
    const unsigned n = unsigned(a.n);
    switch (a.g.nh) {
    case 2: hipLaunchKernelGGL((k_init<F, 2, 64>), dim3(n), dim3(64), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_init<F, 4, 64>), dim3(n), dim3(64), 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_init<F, 6, 256>), dim3(n), dim3(256), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_init<F, 8, 256>), dim3(n), dim3(256), 0, st, a); break;
    case 12: hipLaunchKernelGGL((k_init<F, 12, 576>), dim3(n), dim3(576), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename F>
hipError_t moments_dispatch(const void *f, double *out, int64_t n, const VelGrid &g, hipStream_t st) {
    const F *p = static_cast<const F *>(f);
    const unsigned nb = unsigned(n);
    switch (g.nh) {
    case 2: hipLaunchKernelGGL((k_moments<F, 2, 64>), dim3(nb), dim3(64), 0, st, p, out, n, g); break;
    case 4: hipLaunchKernelGGL((k_moments<F, 4, 64>), dim3(nb), dim3(64), 0, st, p, out, n, g); break;
    case 6: hipLaunchKernelGGL((k_moments<F, 6, 256>), dim3(nb), dim3(256), 0, st, p, out, n, g); break;
    case 8: hipLaunchKernelGGL((k_moments<F, 8, 256>), dim3(nb), dim3(256), 0, st, p, out, n, g); break;
    case 12: hipLaunchKernelGGL((k_moments<F, 12, 256>), dim3(nb), dim3(256), 0, st, p, out, n, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename F>
hipError_t wall_den_dispatch(const void *m1, double *den, const VelGrid &g, hipStream_t st) {
    const F *p = static_cast<const F *>(m1);
    switch (g.nh) {
    case 2: hipLaunchKernelGGL((k_wall_den<F, 2>), dim3(1), dim3(256), 0, st, p, den, g); break;
    case 4: hipLaunchKernelGGL((k_wall_den<F, 4>), dim3(1), dim3(256), 0, st, p, den, g); break;
    case 6: hipLaunchKernelGGL((k_wall_den<F, 6>), dim3(1), dim3(256), 0, st, p, den, g); break;
    case 8: hipLaunchKernelGGL((k_wall_den<F, 8>), dim3(1), dim3(256), 0, st, p, den, g); break;
    case 12: hipLaunchKernelGGL((k_wall_den<F, 12>), dim3(1), dim3(256), 0, st, p, den, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool have_kernel(bool fp64, int nh, int threads) {
    (void)fp64;
#define X(NH, T) \
    if (nh == NH && threads == T) return true;
    DVM_STEP_CONFIGS(X)
#undef X
    return false;
}

int default_threads(bool fp64, int nh) { return fp64 ? default_threads_t<double>(nh) : default_threads_t<float>(nh); }

hipError_t launch_step(bool fp64, const StepArgs &a, const StepConfig &cfg, hipStream_t st) {
    return fp64 ? step_dispatch<double>(a.g.nh, cfg.threads, a, st) : step_dispatch<float>(a.g.nh, cfg.threads, a, st);
}

hipError_t launch_init(bool fp64, const InitArgs &a, hipStream_t st) {
    return fp64 ? init_dispatch<double>(a, st) : init_dispatch<float>(a, st);
}

hipError_t launch_moments(bool fp64, const void *f, double *out, int64_t n, const VelGrid &g, hipStream_t st) {
    return fp64 ? moments_dispatch<double>(f, out, n, g, st) : moments_dispatch<float>(f, out, n, g, st);
}

hipError_t launch_wall_den(bool fp64, const void *m1, double *den, const VelGrid &g, hipStream_t st) {
    return fp64 ? wall_den_dispatch<double>(m1, den, g, st) : wall_den_dispatch<float>(m1, den, g, st);
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
