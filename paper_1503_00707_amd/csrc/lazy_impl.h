// lazy_impl.h -- the streaming ("deferred collision") engine of the DVM-BGK
// step, instantiated per storage precision in kernels_f32.hip / kernels_f64.hip.
//
// State.  Instead of f^n the engine stores f*^n, the state right after the
// transport of step n-1, and per cell the table of the BGK relaxation that
// turns it into f^n (the collision of section 4 toward the eq. 6 corrected
// Maxwellian of the cell's own moments):
//     f^n_i = e f*_i + G_x[kx] G_y[ky] G_z[kz] (P_x[kx] + P_y[ky] + P_z[kz]),
// record per cell: (G, P) per axis and node, e, and the diffuse-wall densities
// of its wall faces.  An identity record (G = P = 0, e = 1) means f = f*.
// The step is the same Lie splitting as the fused engine, the collision being
// applied when a value is read (same arithmetic as the eager relaxation):
//
//   k_unit   one workgroup per (cell, octant) block of NH^3 values.  The
//            octant fixes the three upwind faces, so every branch is
//            workgroup-uniform.  It reads the cell's block and the upwind
//            neighbours' blocks, relaxes each with its owner's table, applies
//            the upwind transport of eq. 2, writes f*^{n+1} and the block's
//            FP64 partial moments.  Workgroup w handles octant w % 8: the
//            hardware deals workgroups to the 8 XCDs round-robin, so each XCD
//            streams one octant in Morton cell order and the neighbour blocks
//            it reads are the blocks its own recent units loaded (L2 hits).
//   k_tables one workgroup per cell: sums the 8 partials in a fixed order,
//            builds the corrected Maxwellian of the moments (maxwell_solve),
//            writes the cell's table, its moments and the wall densities.
//
// Thread map inside a unit: thread t < NH^2 owns (ay, az) = (t / NH, t % NH)
// and loops over ax, so its y/z record factors are loaded once per unit and
// the x factors are workgroup-uniform; 64 lanes read 256 contiguous bytes.
#pragma once

#include "step_impl.h"

namespace dvm {
namespace impl {

// table record: (G,P) for axis b, node k at 2*(b*N + k); e at 6N; rho_w[f] at 6N+1+f
template <int NH>
struct TabLayout {
    static constexpr int N = 2 * NH;
    static constexpr int kE = 6 * N;
    static constexpr int kRhoW = 6 * N + 1;
    static constexpr int kStride = 6 * N + 8;
};


// The cell record read with runtime face indices (scalar loads from memory).
struct CellPtr {
    cuint32_t *p;
    __device__ __forceinline__ CellPtr(const DevCell *cells, int64_t c)
        : p(as_const_space(reinterpret_cast<const uint32_t *>(cells + c))) {}
    __device__ __forceinline__ int type(int f) const { return (p[24 + (f >> 2)] >> (8 * (f & 3))) & 0xff; }
    __device__ __forceinline__ int level() const { return (p[25] >> 16) & 0xff; }
    __device__ __forceinline__ int32_t nbr(int f, int k) const { return int32_t(p[4 * f + k]); }
};

struct UnitArgs {
    const void *f_in;
    void *f_out;
    const void *tab;        // [n][stride] records of f_in
    double *partials;       // [8][n][5] sums (1, xi, |xi|^2/2) f* per octant, no weight
    const DevCell *cells;
    const void *ghost_in;
    const void *wall_m1;
    const void *null_rec;   // an identity record (G = P = 0, e = 1)
    int64_t n_cells;
    double dt;
    double h0;
    VelGrid g;
};

// The relaxed value of one upwind source for the slots (ay, az) x all ax:
//   f = e f* + G_x[kx] (G_y[ky] G_z[kz]) (P_x[kx] + (P_y[ky] + P_z[kz])).
// x factors are workgroup-uniform (scalar loads), y/z factors per lane.
template <typename F, int NH>
struct RecView {
    cF<F> *rec;  // x factors and e: uniform, scalar loads
    F gyz, pyz, e;
    int sx;
    __device__ __forceinline__ RecView(const F *r, int ky, int kz, int sx_)
        : rec(as_const_space(r)), sx(sx_) {
        constexpr int N = 2 * NH;
        gyz = r[2 * (N + ky)] * r[2 * (2 * N + kz)];
        pyz = r[2 * (N + ky) + 1] + r[2 * (2 * N + kz) + 1];
        e = rec[6 * N];
    }
    __device__ __forceinline__ F apply(int ax, F fstar) const {
        const int kx = sx ? NH + ax : NH - 1 - ax;
        return e * fstar + (rec[2 * kx] * gyz) * (rec[2 * kx + 1] + pyz);
    }
};

// TRANSPORT = false: partial moments of the relaxed state only (no store).
// Launch TL = ceil64(NH^2) threads per (cell, octant) unit; thread t < NH^2
// owns (ay, az) = (t / NH, t % NH) and all NH values of ax.
template <typename F, int NH, int TL, int WPE, bool TRANSPORT, bool NT>
__global__ __launch_bounds__(TL) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_unit(UnitArgs a) {
    constexpr int B = NH * NH * NH;
    constexpr int P2 = NH * NH;
    constexpr int64_t NV = 8 * B;
    using TLy = TabLayout<NH>;
    static_assert(P2 <= TL && TL % 64 == 0, "unit shape");
    constexpr uint32_t kRow = uint32_t(NV * sizeof(F));
    __shared__ double red[(TL / 64) * 5];

    // 2D grid (a dispatch counts work-items in 32 bits): gridDim.x is a
    // multiple of 8, so the linear workgroup id and blockIdx.x agree mod 8
    const uint32_t w = blockIdx.x + blockIdx.y * gridDim.x;
    const int o = int(w & 7u);
    const int64_t c = __builtin_amdgcn_readfirstlane(w >> 3);
    if (c >= a.n_cells) return;
    const int sg[3] = {o >> 2, (o >> 1) & 1, o & 1};
    const CellPtr cell(a.cells, c);
    const F *fin = static_cast<const F *>(a.f_in);
    const F *tab = static_cast<const F *>(a.tab);
    const int tid = threadIdx.x;
    const bool act = tid < P2;
    const int pp = act ? tid : 0;
    const int ay = pp / NH, az = pp % NH;
    const int ky = sg[1] ? NH + ay : NH - 1 - ay;
    const int kz = sg[2] ? NH + az : NH - 1 - az;
    const uint32_t voff = uint32_t(pp) * sizeof(F);
    const uint32_t obase = uint32_t(o * B);
    auto soff = [&](int ax) { return uint32_t((obase + ax * P2) * sizeof(F)); };

    const F *own_rec = tab + c * TLy::kStride;
    const RecView<F, NH> r0(own_rec, ky, kz, sg[0]);
    const Rsrc own = rsrc(fin + c * NV, kRow);
    F fv[NH];
#pragma unroll
    for (int ax = 0; ax < NH; ++ax) fv[ax] = r0.apply(ax, bld<F>(own, voff, soff(ax)));

    if (TRANSPORT) {
        const double dth = a.dt / (a.h0 / double(1 << cell.level()));
        const F nuy = F(dth * ((ay + 0.5) * a.g.dv[1])), nuz = F(dth * ((az + 0.5) * a.g.dv[2]));
        // main pass: one row and one record per axis, no branch in the value loop.
        // FINER and WALL faces read an empty row here and are added below.
        int uf[3], ty[3];
        const F *rowp[3];
        const F *recp[3];
        uint32_t bytes[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            uf[b] = 2 * b + (sg[b] ? 0 : 1);  // a positive component enters through the low face
            ty[b] = cell.type(uf[b]);
            rowp[b] = fin + c * NV;  // OUTFLOW: the cell's own relaxed value
            recp[b] = own_rec;
            bytes[b] = kRow;
            if (ty[b] == DVM_FACE_SAME || ty[b] == DVM_FACE_COARSER) {
                const int64_t nb = cell.nbr(uf[b], 0);
                rowp[b] = fin + nb * NV;
                recp[b] = tab + nb * TLy::kStride;
            } else if (ty[b] == DVM_FACE_INFLOW) {
                rowp[b] = static_cast<const F *>(a.ghost_in);
                recp[b] = static_cast<const F *>(a.null_rec);
            } else if (ty[b] == DVM_FACE_FINER || ty[b] == DVM_FACE_WALL) {
                recp[b] = static_cast<const F *>(a.null_rec);
                bytes[b] = 0;
            }
        }
        F acc[NH];
#pragma unroll
        for (int ax = 0; ax < NH; ++ax) acc[ax] = F(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const RecView<F, NH> rv(recp[b], ky, kz, sg[0]);
            const Rsrc rr = rsrc(rowp[b], bytes[b]);
#pragma unroll
            for (int ax = 0; ax < NH; ++ax) {
                const F up = rv.apply(ax, bld<F>(rr, voff, soff(ax)));
                const F nu = b == 0 ? F(dth * ((ax + 0.5) * a.g.dv[0])) : b == 1 ? nuy : nuz;
                acc[ax] += nu * (fv[ax] - up);
            }
        }
        // correction for FINER (mean of four relaxed finer rows) and WALL
        // (rho_w times the wall Maxwellian) faces: workgroup-uniform branches
#pragma nounroll
        for (int b = 0; b < 3; ++b) {
            const int t = ty[b];
            if (t != DVM_FACE_FINER && t != DVM_FACE_WALL) continue;
            const int f = uf[b];
#pragma nounroll
            for (int k = 0; k < (t == DVM_FACE_FINER ? 4 : 1); ++k) {
                const int64_t nb = t == DVM_FACE_FINER ? cell.nbr(f, k) : 0;
                const RecView<F, NH> rv(t == DVM_FACE_FINER ? tab + nb * TLy::kStride
                                                            : static_cast<const F *>(a.null_rec),
                                        ky, kz, sg[0]);
                const Rsrc rr = rsrc(t == DVM_FACE_FINER ? fin + nb * NV : static_cast<const F *>(a.wall_m1), kRow);
                const F sc = t == DVM_FACE_FINER ? F(0.25) : own_rec[TLy::kRhoW + f];
#pragma unroll
                for (int ax = 0; ax < NH; ++ax) {
                    const F up = sc * rv.apply(ax, bld<F>(rr, voff, soff(ax)));
                    const F nu = b == 0 ? F(dth * ((ax + 0.5) * a.g.dv[0])) : b == 1 ? nuy : nuz;
                    acc[ax] -= nu * up;  // the main pass counted this source as 0
                }
            }
        }
#pragma unroll
        for (int ax = 0; ax < NH; ++ax) fv[ax] -= acc[ax];
        if (act) {
            const Rsrc out = rsrc(static_cast<F *>(a.f_out) + c * NV, kRow);
#pragma unroll
            for (int ax = 0; ax < NH; ++ax) bst<F, NT ? kAuxNT : 0>(out, voff, soff(ax), fv[ax]);
        }
    }

    // FP64 partial moments of the block (signs of the octant applied at the end)
    double s0 = 0.0, sx = 0.0, sxx = 0.0;
    if (act) {
#pragma unroll
        for (int ax = 0; ax < NH; ++ax) {
            const double xa = (ax + 0.5) * a.g.dv[0];
            const double d = double(fv[ax]);
            s0 += d;
            sx += xa * d;
            sxx += xa * xa * d;
        }
    }
    const double ya = (ay + 0.5) * a.g.dv[1], za = (az + 0.5) * a.g.dv[2];
    const double xs = sg[0] ? 1.0 : -1.0, ys = sg[1] ? 1.0 : -1.0, zs = sg[2] ? 1.0 : -1.0;
    double m[5] = {s0, xs * sx, ys * ya * s0, zs * za * s0, 0.5 * (sxx + (ya * ya + za * za) * s0)};
    block_sum<TL, 5>(m, red);
    if (tid == 0) {
        double *pq = a.partials + (int64_t(o) * a.n_cells + c) * 5;
        for (int k = 0; k < 5; ++k) pq[k] = m[k];
    }
}

struct TableArgs {
    const double *partials;  // [8][n][5]
    void *tab;               // [n][stride]
    double *mom;             // [5][n] or NULL
    const DevCell *cells;
    const double *wall_den;  // [6]
    int *flag;
    int64_t n_cells;
    double dt;
    VelGrid g;
    int collide;             // 0: identity records (no relaxation pending)
    int collision;           // DVM_COLL_*
    int tau_mode;
    double tau_or_kn;
};

// Per cell: moments from the partials, the relaxation record for the next
// transport, and the wall densities (zero net mass flux through each wall
// face for the relaxed state: rho_w = sum_{xi.n>0} (xi.n) f / den_f, the sum
// split into e * (from the partials of f*) + (separable sum of the table).
template <typename F, int NH>
__global__ __launch_bounds__(64) void k_tables(TableArgs a) {
    using TLy = TabLayout<NH>;
    constexpr int N = 2 * NH;
    __shared__ MaxwellSmem<F, NH> sm;
    __shared__ double gp[3][N][2];  // FP64 G, P of the record
    const int64_t c = blockIdx.x;
    const int64_t n = a.n_cells;
    double m[5] = {0, 0, 0, 0, 0};
    for (int o = 0; o < 8; ++o)
        for (int k = 0; k < 5; ++k) m[k] += a.partials[(int64_t(o) * n + c) * 5 + k];
    const double w = a.g.w;
    const double rho = w * m[0];
    const double u[3] = {w * m[1] / rho, w * m[2] / rho, w * m[3] / rho};
    const double E = w * m[4];
    const double Tt = (2.0 * E / rho - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / 3.0;
    const bool bad = !(rho > 0.0) || !(Tt > 0.0);
    if (threadIdx.x == 0) {
        if (a.mom) {
            a.mom[c] = rho;
            a.mom[n + c] = w * m[1];
            a.mom[2 * n + c] = w * m[2];
            a.mom[3 * n + c] = w * m[3];
            a.mom[4 * n + c] = E;
        }
        if (bad) *a.flag = 1;
    }
    const bool relax = a.collide && !bad && a.collision != DVM_COLL_OFF;
    double e = 1.0;
    if (relax) {
        const double tau = a.tau_mode == DVM_TAU_HS ? a.tau_or_kn / (rho * sqrt(Tt)) : a.tau_or_kn;
        double mfac;
        if (a.collision == DVM_COLL_EULER) {
            e = 1.0 - a.dt / tau;
            mfac = a.dt / tau;
        } else {
            e = exp(-a.dt / tau);
            mfac = -expm1(-a.dt / tau);
        }
        maxwell_solve<F, NH, 64>(sm, rho, u, Tt, a.g);
        for (int j = threadIdx.x; j < 3 * N; j += 64) {
            const int b = j / N, k = j % N;
            const double cc = sm.c[b][k];
            gp[b][k][0] = b == 0 ? sm.g[b][k] * sm.C * mfac : sm.g[b][k];
            gp[b][k][1] = b == 0 ? 1.0 + sm.d[0] + sm.d[1] * cc + sm.d[4] * cc * cc : sm.d[1 + b] * cc + sm.d[4] * cc * cc;
        }
    } else {
        for (int j = threadIdx.x; j < 3 * N; j += 64) {
            const int b = j / N, k = j % N;
            gp[b][k][0] = 0.0;
            gp[b][k][1] = 0.0;
        }
    }
    __syncthreads();
    F *rec = static_cast<F *>(a.tab) + c * TLy::kStride;
    for (int j = threadIdx.x; j < 6 * N; j += 64) rec[j] = F(gp[j / (2 * N)][(j / 2) % N][j & 1]);
    if (threadIdx.x == 0) {
        rec[TLy::kE] = F(e);
        const uint32_t *cw = reinterpret_cast<const uint32_t *>(a.cells + c);
        const uint32_t w25 = cw[25];
#pragma nounroll
        for (int f = 0; f < 6; ++f) {
            const int tyf = f < 4 ? (cw[24] >> (8 * f)) & 0xff : (w25 >> (8 * (f - 4))) & 0xff;
            double rw = 0.0;
            if (tyf == DVM_FACE_WALL) {
                const int axis = f >> 1, side = f & 1;
                // leaving: velocities with sign bit == side along the axis
                double num = 0.0;
                for (int o = 0; o < 8; ++o) {
                    const int sb = axis == 0 ? (o >> 2) : axis == 1 ? ((o >> 1) & 1) : (o & 1);
                    if (sb == side) num += (side ? 1.0 : -1.0) * a.partials[(int64_t(o) * n + c) * 5 + 1 + axis];
                }
                num *= e;
                if (relax) {
                    // sum over the leaving half of |xi_axis| Gx Gy Gz (Px + Py + Pz), separable
                    double A1 = 0, A2 = 0, B1[3] = {0, 0, 0}, B2[3] = {0, 0, 0};
#pragma unroll
                    for (int b = 0; b < 3; ++b)
#pragma nounroll
                        for (int k = 0; k < N; ++k) {
                            B1[b] += gp[b][k][0];
                            B2[b] += gp[b][k][0] * gp[b][k][1];
                        }
#pragma nounroll
                    for (int k = side ? NH : 0; k < (side ? N : NH); ++k) {
                        const double xa = (k < NH ? NH - 1 - k : k - NH) + 0.5;
                        A1 += xa * a.g.dv[axis] * gp[axis][k][0];
                        A2 += xa * a.g.dv[axis] * gp[axis][k][0] * gp[axis][k][1];
                    }
                    const int b1 = (axis + 1) % 3, b2 = (axis + 2) % 3;
                    num += A2 * B1[b1] * B1[b2] + A1 * (B2[b1] * B1[b2] + B1[b1] * B2[b2]);
                }
                rw = num / a.wall_den[f];
            }
            rec[TLy::kRhoW + f] = F(rw);
        }
    }
}

// canonical index (kx*N + ky)*N + kz  <-  relaxed internal state
template <typename F, int NH>
__global__ __launch_bounds__(256) void k_canon_relaxed(const F *fstar, const F *tab, F *dst) {
    using TLy = TabLayout<NH>;
    constexpr int64_t B = NH * NH * NH, NV = 8 * B, N = 2 * NH;
    const int64_t c = blockIdx.x;
    const F *rec = tab + c * TLy::kStride;
    const F e = rec[TLy::kE];
    for (int64_t v = threadIdx.x; v < NV; v += 256) {
        const int64_t o = v / B, s = v % B;
        const int64_t ax = s / (NH * NH), ay = (s / NH) % NH, az = s % NH;
        const int64_t kx = (o >> 2) ? NH + ax : NH - 1 - ax;
        const int64_t ky = ((o >> 1) & 1) ? NH + ay : NH - 1 - ay;
        const int64_t kz = (o & 1) ? NH + az : NH - 1 - az;
        const F M = (rec[2 * kx] * (rec[2 * (N + ky)] * rec[2 * (2 * N + kz)])) *
                    (rec[2 * kx + 1] + (rec[2 * (N + ky) + 1] + rec[2 * (2 * N + kz) + 1]));
        dst[c * NV + (kx * N + ky) * N + kz] = e * fstar[c * NV + v] + M;
    }
}

// f* := relaxed state, record := identity (wall densities kept: the state is unchanged)
template <typename F, int NH>
__global__ __launch_bounds__(256) void k_materialize(F *fstar, F *tab) {
    using TLy = TabLayout<NH>;
    constexpr int64_t B = NH * NH * NH, NV = 8 * B, N = 2 * NH;
    const int64_t c = blockIdx.x;
    F *rec = tab + c * TLy::kStride;
    const F e = rec[TLy::kE];
    for (int64_t v = threadIdx.x; v < NV; v += 256) {
        const int64_t o = v / B, s = v % B;
        const int64_t ax = s / (NH * NH), ay = (s / NH) % NH, az = s % NH;
        const int64_t kx = (o >> 2) ? NH + ax : NH - 1 - ax;
        const int64_t ky = ((o >> 1) & 1) ? NH + ay : NH - 1 - ay;
        const int64_t kz = (o & 1) ? NH + az : NH - 1 - az;
        const F M = (rec[2 * kx] * (rec[2 * (N + ky)] * rec[2 * (2 * N + kz)])) *
                    (rec[2 * kx + 1] + (rec[2 * (N + ky) + 1] + rec[2 * (2 * N + kz) + 1]));
        fstar[c * NV + v] = e * fstar[c * NV + v] + M;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < 6 * N; j += 256) rec[j] = F(0);
    if (threadIdx.x == 0) rec[TLy::kE] = F(1);
}

// identity records: no relaxation pending, no wall density yet
template <typename F, int NH>
__global__ __launch_bounds__(64) void k_identity(F *tab) {
    using TLy = TabLayout<NH>;
    F *rec = tab + int64_t(blockIdx.x) * TLy::kStride;
    for (int j = threadIdx.x; j < TLy::kStride; j += 64) rec[j] = j == TLy::kE ? F(1) : F(0);
}

// moments [5][n] from the partials
template <int U>
__global__ __launch_bounds__(256) void k_sum_partials(const double *partials, double *out, int64_t n, double w) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= n) return;
    double m[5] = {0, 0, 0, 0, 0};
    for (int o = 0; o < 8; ++o)
        for (int k = 0; k < 5; ++k) m[k] += partials[(int64_t(o) * n + c) * 5 + k];
    for (int k = 0; k < 5; ++k) out[k * n + c] = w * m[k];
}

// Partial moments of the relaxed state (no transport): one shape per N.
#define DVM_UNIT_CONFIGS(X) \
    X(2, 64, 8)             \
    X(4, 64, 8)             \
    X(6, 64, 8)             \
    X(8, 64, 8)             \
    X(12, 192, 5)

template <typename F>
hipError_t unit_dispatch(const UnitArgs &a, hipStream_t st) {
    const int64_t units = 8 * a.n_cells;
    const unsigned gx = unsigned(units < 8 * 16384 ? units : 8 * 16384);
    const dim3 grid(gx, unsigned((units + gx - 1) / gx));
#define X(NH, TL, W)                                                                              \
    if (a.g.nh == NH) {                                                                           \
        hipLaunchKernelGGL((k_unit<F, NH, TL, W, false, false>), grid, dim3(TL), 0, st, a);       \
        return hipGetLastError();                                                                 \
    }
    DVM_UNIT_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

template <typename F>
hipError_t tables_dispatch(const TableArgs &a, hipStream_t st) {
    const dim3 grid(unsigned(a.n_cells));
    switch (a.g.nh) {
    case 2: hipLaunchKernelGGL((k_tables<F, 2>), grid, dim3(64), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_tables<F, 4>), grid, dim3(64), 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_tables<F, 6>), grid, dim3(64), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_tables<F, 8>), grid, dim3(64), 0, st, a); break;
    case 12: hipLaunchKernelGGL((k_tables<F, 12>), grid, dim3(64), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename F>
hipError_t canon_relaxed_dispatch(const void *fstar, const void *tab, void *dst, int64_t n, int nh, hipStream_t st) {
    const F *p = static_cast<const F *>(fstar);
    const F *t = static_cast<const F *>(tab);
    F *d = static_cast<F *>(dst);
    switch (nh) {
    case 2: hipLaunchKernelGGL((k_canon_relaxed<F, 2>), dim3(unsigned(n)), dim3(256), 0, st, p, t, d); break;
    case 4: hipLaunchKernelGGL((k_canon_relaxed<F, 4>), dim3(unsigned(n)), dim3(256), 0, st, p, t, d); break;
    case 6: hipLaunchKernelGGL((k_canon_relaxed<F, 6>), dim3(unsigned(n)), dim3(256), 0, st, p, t, d); break;
    case 8: hipLaunchKernelGGL((k_canon_relaxed<F, 8>), dim3(unsigned(n)), dim3(256), 0, st, p, t, d); break;
    case 12: hipLaunchKernelGGL((k_canon_relaxed<F, 12>), dim3(unsigned(n)), dim3(256), 0, st, p, t, d); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename F>
hipError_t identity_dispatch(void *tab, int64_t n, int nh, hipStream_t st) {
    F *t = static_cast<F *>(tab);
    switch (nh) {
    case 2: hipLaunchKernelGGL((k_identity<F, 2>), dim3(unsigned(n)), dim3(64), 0, st, t); break;
    case 4: hipLaunchKernelGGL((k_identity<F, 4>), dim3(unsigned(n)), dim3(64), 0, st, t); break;
    case 6: hipLaunchKernelGGL((k_identity<F, 6>), dim3(unsigned(n)), dim3(64), 0, st, t); break;
    case 8: hipLaunchKernelGGL((k_identity<F, 8>), dim3(unsigned(n)), dim3(64), 0, st, t); break;
    case 12: hipLaunchKernelGGL((k_identity<F, 12>), dim3(unsigned(n)), dim3(64), 0, st, t); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

inline int tab_stride(int nh) { return 12 * nh + 8; }

template <typename F>
hipError_t materialize_dispatch(void *fstar, void *tab, int64_t n, int nh, hipStream_t st) {
    F *p = static_cast<F *>(fstar);
    F *t = static_cast<F *>(tab);
    switch (nh) {
    case 2: hipLaunchKernelGGL((k_materialize<F, 2>), dim3(unsigned(n)), dim3(256), 0, st, p, t); break;
    case 4: hipLaunchKernelGGL((k_materialize<F, 4>), dim3(unsigned(n)), dim3(256), 0, st, p, t); break;
    case 6: hipLaunchKernelGGL((k_materialize<F, 6>), dim3(unsigned(n)), dim3(256), 0, st, p, t); break;
    case 8: hipLaunchKernelGGL((k_materialize<F, 8>), dim3(unsigned(n)), dim3(256), 0, st, p, t); break;
    case 12: hipLaunchKernelGGL((k_materialize<F, 12>), dim3(unsigned(n)), dim3(256), 0, st, p, t); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace impl
}  // namespace dvm
