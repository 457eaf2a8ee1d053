// sweep_impl.h -- persistent transport sweep of the deferred-collision engine.
//
// The same step as k_unit (relax each source with its owner's record, upwind
// transport of eq. 2, store f*, FP64 partial moments per (cell, octant)), but
// as a persistent grid: workgroup w serves octant o = w % 8 (so each XCD
// streams one octant) and cells j, j + P, j + 2P, ... of it (j = w / 8, P
// workgroups per octant), so at any time the P workgroups of an XCD work on a
// window of about P consecutive Morton cells and the upwind blocks they read
// are blocks that the window loaded moments before (L2 hits).
//
// Software pipeline: while a unit is computed, the loads of the next unit of
// the same workgroup (its own block, the three upwind blocks and the four
// relaxation records) are already in flight, so the latency of the dependent
// chain cell record -> neighbour index -> data is hidden behind the
// arithmetic of the previous unit.  Records are staged through LDS: the x
// factors are then workgroup-uniform broadcast reads, the y/z factors one
// read per lane.
#pragma once

#include "lazy_impl.h"

namespace dvm {
namespace impl {

template <int NH>
struct SweepShape {
    static constexpr int P2 = NH * NH;
    static constexpr int T = (P2 + 63) / 64 * 64;  // one lane per (ay, az)
    static constexpr int RH = 2 * NH;               // (G, P) pairs of one axis half
    static constexpr int RS = 3 * RH + 2;           // staged floats per source: x, y, z halves, e, pad
    static constexpr int RALL = 4 * RS;             // own + three upwind sources
    static constexpr int RL = (RALL + T - 1) / T;   // staging loads per thread
};

// Uniform description of one unit (SGPRs).  Records are addressed by cell
// index; index n_cells is the identity record (no relaxation).
template <typename F>
struct SweepMeta {
    int64_t c;
    int level;
    int ty[3];
    const F *row[3];
    uint32_t bytes[3];
    uint32_t ri[3];  // record index of each upwind source
};

// Values of one unit in flight (VGPRs).
template <typename F, int NH>
struct SweepStage {
    F own[NH];
    F up[3][NH];
    F rr[SweepShape<NH>::RL];
};

template <typename F, int NH>
__device__ __forceinline__ void sweep_meta(const UnitArgs &a, int64_t c, const int (&sg)[3], SweepMeta<F> &m) {
    constexpr int64_t NV = 8 * NH * NH * NH;
    constexpr uint32_t kRow = uint32_t(NV * sizeof(F));
    const F *fin = static_cast<const F *>(a.f_in);
    const CellPtr cell(a.cells, c);
    const uint32_t null_ri = uint32_t(a.n_cells);
    m.c = c;
    m.level = cell.level();
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int f = 2 * b + (sg[b] ? 0 : 1);  // a positive component enters through the low face
        const int t = cell.type(f);
        m.ty[b] = t;
        m.row[b] = fin + c * NV;  // OUTFLOW: the cell's own relaxed value
        m.ri[b] = uint32_t(c);
        m.bytes[b] = kRow;
        if (t == DVM_FACE_SAME || t == DVM_FACE_COARSER) {
            const int64_t nb = cell.nbr(f, 0);
            m.row[b] = fin + nb * NV;
            m.ri[b] = uint32_t(nb);
        } else if (t == DVM_FACE_INFLOW) {
            m.row[b] = static_cast<const F *>(a.ghost_in);
            m.ri[b] = null_ri;
        } else if (t == DVM_FACE_FINER || t == DVM_FACE_WALL) {
            m.ri[b] = null_ri;
            m.bytes[b] = 0;  // added by the correction pass
        }
    }
}

// Offset inside a record of staged element r of one source.  The staged
// copy of an axis half is in |xi| order: element 2a + q (q = 0: G, 1: P) is
// the node at distance a from the centre on the octant's side, so that the
// reads of the transport pass have compile-time offsets.  The last two
// elements are e (and a pad that re-reads it).
template <int NH>
__device__ __forceinline__ int sweep_rec_offset(int r, int sx, int sy, int sz) {
    using SS = SweepShape<NH>;
    using TLy = TabLayout<NH>;
    constexpr int N = 2 * NH;
    if (r >= 3 * SS::RH) return TLy::kE;
    const int seg = r / SS::RH, within = r - seg * SS::RH;
    const int s = seg == 0 ? sx : seg == 1 ? sy : sz;
    const int a = within >> 1, q = within & 1;
    const int k = s ? NH + a : NH - 1 - a;
    return 2 * (seg * N + k) + q;
}

template <typename F, int NH, int WPE, bool NT>
__global__ __launch_bounds__(SweepShape<NH>::T) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_sweep(
    UnitArgs a, int per_octant) {
    using SS = SweepShape<NH>;
    using TLy = TabLayout<NH>;
    constexpr int T = SS::T;
    constexpr int B = NH * NH * NH;
    constexpr int P2 = NH * NH;
    constexpr int64_t NV = 8 * B;
    constexpr uint32_t kRow = uint32_t(NV * sizeof(F));
    __shared__ __attribute__((aligned(16))) F recs[2][SS::RALL];
    __shared__ __attribute__((aligned(16))) F recf[SS::RALL];  // records of the four finer cells
    __shared__ double red[(T / 64) * 5];

    const int o = int(blockIdx.x & 7u);
    const int64_t j = blockIdx.x >> 3;
    const int64_t P = per_octant;
    if (j >= a.n_cells) return;
    const int sx = o >> 2, sy = (o >> 1) & 1, sz = o & 1;
    const int sg[3] = {sx, sy, sz};
    const F *fin = static_cast<const F *>(a.f_in);
    const int tid = threadIdx.x;
    const bool act = tid < P2;
    const int pp = act ? tid : 0;
    const int ay = pp / NH, az = pp % NH;
    const uint32_t voff = uint32_t(pp) * sizeof(F);
    const uint32_t obase = uint32_t(o * B);
    auto soff = [&](int ax) { return uint32_t((obase + ax * P2) * sizeof(F)); };
    // the records (and the identity record after them) through one descriptor
    const Rsrc rtab = rsrc(a.tab, uint32_t((a.n_cells + 1) * TLy::kStride * int64_t(sizeof(F))));
    const Rsrc rtab0 = rsrc(a.tab, 0u);
    const double dt_h0 = a.dt / a.h0;
    // staged record elements of this thread: source and byte offset in the record
    int rsel[SS::RL];
    uint32_t roff[SS::RL];
#pragma unroll
    for (int l = 0; l < SS::RL; ++l) {
        const int el = tid + l * T;
        const int e2 = el < SS::RALL ? el : 0;
        rsel[l] = el < SS::RALL ? e2 / SS::RS : 4;
        roff[l] = uint32_t(sweep_rec_offset<NH>(e2 % SS::RS, sx, sy, sz) * sizeof(F));
    }

    // loads of a unit; live == false issues the same loads through empty
    // descriptors (they return 0 without touching memory), so that every
    // iteration has the same number of loads in flight and the wait for the
    // current unit never has to drain the next one
    auto issue = [&](const SweepMeta<F> &m, bool live, SweepStage<F, NH> &st) {
        const Rsrc own = rsrc(fin + m.c * NV, live ? kRow : 0u);
#pragma unroll
        for (int ax = 0; ax < NH; ++ax) st.own[ax] = bld<F>(own, voff, soff(ax));
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const Rsrc r = rsrc(m.row[b], live ? m.bytes[b] : 0u);
#pragma unroll
            for (int ax = 0; ax < NH; ++ax) st.up[b][ax] = bld<F>(r, voff, soff(ax));
        }
        const Rsrc rt = live ? rtab : rtab0;
        const uint32_t c32 = uint32_t(m.c);
#pragma unroll
        for (int l = 0; l < SS::RL; ++l) {
            const int s = rsel[l];
            const uint32_t ri = s == 0 ? c32 : s == 1 ? m.ri[0] : s == 2 ? m.ri[1] : m.ri[2];
            st.rr[l] = bld<F>(rt, ri * uint32_t(TLy::kStride * sizeof(F)) + roff[l], 0);
        }
    };

    auto compute = [&](const SweepMeta<F> &m, const SweepStage<F, NH> &st, F *R) {
#pragma unroll
        for (int l = 0; l < SS::RL; ++l)
            if (rsel[l] < 4) R[tid + l * T] = st.rr[l];
        __syncthreads();
        const double dth = ldexp(dt_h0, m.level);  // dt / h, exact: h = h0 2^-level
        const F nuy = F(dth * ((ay + 0.5) * a.g.dv[1])), nuz = F(dth * ((az + 0.5) * a.g.dv[2]));
        // x Courant numbers from literal (k + 1/2): no per-ax constants held in registers
        const double dthx = dth * a.g.dv[0];
        F fv[NH], acc[NH];
        {
            const F *Rs = R;
            const F gyz = Rs[SS::RH + 2 * ay] * Rs[2 * SS::RH + 2 * az];
            const F pyz = Rs[SS::RH + 2 * ay + 1] + Rs[2 * SS::RH + 2 * az + 1];
            const F es = Rs[3 * SS::RH];
#pragma unroll
            for (int ax = 0; ax < NH; ++ax) {
                fv[ax] = es * st.own[ax] + (Rs[2 * ax] * gyz) * (Rs[2 * ax + 1] + pyz);
                acc[ax] = F(0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const F *Rs = R + (1 + b) * SS::RS;
            const F gyz = Rs[SS::RH + 2 * ay] * Rs[2 * SS::RH + 2 * az];
            const F pyz = Rs[SS::RH + 2 * ay + 1] + Rs[2 * SS::RH + 2 * az + 1];
            const F es = Rs[3 * SS::RH];
#pragma unroll
            for (int ax = 0; ax < NH; ++ax) {
                const F up = es * st.up[b][ax] + (Rs[2 * ax] * gyz) * (Rs[2 * ax + 1] + pyz);
                const F nu = b == 0 ? F(dthx * (ax + 0.5)) : b == 1 ? nuy : nuz;
                acc[ax] += nu * (fv[ax] - up);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // FINER (mean of four relaxed finer blocks) and WALL (rho_w times the
        // wall Maxwellian) faces, workgroup-uniform branches.  All loads of a
        // face are issued together (one wait), the four finer records are
        // staged through LDS like the main ones.
        const int tys = m.ty[0] | (m.ty[1] << 8) | (m.ty[2] << 16);
#pragma nounroll
        for (int b = 0; b < 3; ++b) {
            const int t = (tys >> (8 * b)) & 0xff;
            if (t != DVM_FACE_FINER && t != DVM_FACE_WALL) continue;
            const int f = 2 * b + (((o >> (2 - b)) & 1) ? 0 : 1);
            const F nub_y = b == 1 ? nuy : nuz;
            if (t == DVM_FACE_WALL) {
                const Rsrc rr = rsrc(a.wall_m1, kRow);
                F wv[NH];
#pragma unroll
                for (int ax = 0; ax < NH; ++ax) wv[ax] = bld<F>(rr, voff, soff(ax));
                const F sc = as_const_space(static_cast<const F *>(a.tab))[m.c * TLy::kStride + TLy::kRhoW + f];
#pragma unroll
                for (int ax = 0; ax < NH; ++ax) {
                    const F nu = b == 0 ? F(dthx * (ax + 0.5)) : nub_y;
                    acc[ax] -= nu * (sc * wv[ax]);  // the main pass counted this source as 0
                }
                continue;
            }
            const CellPtr cell(a.cells, m.c);
            const uint32_t q0 = uint32_t(cell.nbr(f, 0)), q1 = uint32_t(cell.nbr(f, 1));
            const uint32_t q2 = uint32_t(cell.nbr(f, 2)), q3 = uint32_t(cell.nbr(f, 3));
            F rq[SS::RL];
#pragma unroll
            for (int l = 0; l < SS::RL; ++l) {
                const int sl = rsel[l];
                const uint32_t ri = sl == 0 ? q0 : sl == 1 ? q1 : sl == 2 ? q2 : q3;
                rq[l] = bld<F>(rtab, ri * uint32_t(TLy::kStride * sizeof(F)) + roff[l], 0);
            }
#pragma unroll
            for (int l = 0; l < SS::RL; ++l)
                if (rsel[l] < 4) recf[tid + l * T] = rq[l];
            __syncthreads();
            F up[NH];
#pragma unroll
            for (int ax = 0; ax < NH; ++ax) up[ax] = F(0);
            // one finer block at a time: its NH loads in flight together
#pragma nounroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t qk = __builtin_amdgcn_readfirstlane(k == 0 ? q0 : k == 1 ? q1 : k == 2 ? q2 : q3);
                const Rsrc rr = rsrc(fin + int64_t(qk) * NV, kRow);
                F fq[NH];
#pragma unroll
                for (int ax = 0; ax < NH; ++ax) fq[ax] = bld<F>(rr, voff, soff(ax));
                const F *Rs = recf + k * SS::RS;
                const F gyz = Rs[SS::RH + 2 * ay] * Rs[2 * SS::RH + 2 * az];
                const F pyz = Rs[SS::RH + 2 * ay + 1] + Rs[2 * SS::RH + 2 * az + 1];
                const F es = Rs[3 * SS::RH];
#pragma unroll
                for (int ax = 0; ax < NH; ++ax)
                    up[ax] += es * fq[ax] + (Rs[2 * ax] * gyz) * (Rs[2 * ax + 1] + pyz);
            }
#pragma unroll
            for (int ax = 0; ax < NH; ++ax) {
                const F nu = b == 0 ? F(dthx * (ax + 0.5)) : nub_y;
                acc[ax] -= nu * (F(0.25) * up[ax]);  // the main pass counted this source as 0
            }
            __syncthreads();  // recf is reused by the next FINER face
        }
#pragma unroll
        for (int ax = 0; ax < NH; ++ax) fv[ax] -= acc[ax];
        if (act) {
            const Rsrc out = rsrc(static_cast<F *>(a.f_out) + m.c * NV, kRow);
#pragma unroll
            for (int ax = 0; ax < NH; ++ax) bst<F, NT ? kAuxNT : 0>(out, voff, soff(ax), fv[ax]);
        }
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (act) {
#pragma unroll
            for (int ax = 0; ax < NH; ++ax) {
                const double k = ax + 0.5;  // |xi_x| / dv_x
                const double d = double(fv[ax]);
                s0 += d;
                s1 += k * d;
                s2 += (k * k) * d;
            }
        }
        s1 *= a.g.dv[0];
        s2 *= a.g.dv[0] * a.g.dv[0];
        const double ya = (ay + 0.5) * a.g.dv[1], za = (az + 0.5) * a.g.dv[2];
        const double xs = sx ? 1.0 : -1.0, ys = sy ? 1.0 : -1.0, zs = sz ? 1.0 : -1.0;
        double mm[5] = {s0, xs * s1, ys * ya * s0, zs * za * s0, 0.5 * (s2 + (ya * ya + za * za) * s0)};
        block_sum<T, 5>(mm, red);
        if (tid == 0) {
            double *pq = a.partials + (int64_t(o) * a.n_cells + m.c) * 5;
            for (int k = 0; k < 5; ++k) pq[k] = mm[k];
        }
    };

    SweepMeta<F> mA, mB;
    SweepStage<F, NH> sA, sB;
    const int64_t last = a.n_cells - 1;
    int64_t cA = j;
    sweep_meta<F, NH>(a, cA, sg, mA);
    issue(mA, true, sA);
    int64_t cB = cA + P;
    for (;;) {
        sweep_meta<F, NH>(a, cB < last ? cB : last, sg, mB);
        issue(mB, cB <= last, sB);
        __builtin_amdgcn_sched_barrier(0);
        compute(mA, sA, recs[0]);
        if (cB > last) break;
        cA = cB + P;
        sweep_meta<F, NH>(a, cA < last ? cA : last, sg, mA);
        issue(mA, cA <= last, sA);
        __builtin_amdgcn_sched_barrier(0);
        compute(mB, sB, recs[1]);
        if (cA > last) break;
        cB = cA + P;
    }
}

// (NH, WG per CU, waves per EU of that occupancy)
#define DVM_SWEEP_CONFIGS(X) \
    X(2, 8, 2)               \
    X(4, 8, 2)               \
    X(6, 8, 2)               \
    X(8, 8, 2)               \
    X(12, 2, 2)              \
    X(12, 3, 3)

template <typename F>
hipError_t sweep_dispatch(const UnitArgs &a, int wg_per_cu, int n_cu, bool nt, hipStream_t st) {
#define X(NH, K, W)                                                                                       \
    if (a.g.nh == NH && (wg_per_cu == 0 || wg_per_cu == K)) {                                            \
        const int per_octant = ((n_cu + 7) / 8) * K;                                                      \
        const dim3 grid(unsigned(8 * per_octant)), blk(SweepShape<NH>::T);                               \
        if (nt) hipLaunchKernelGGL((k_sweep<F, NH, W, true>), grid, blk, 0, st, a, per_octant);          \
        else hipLaunchKernelGGL((k_sweep<F, NH, W, false>), grid, blk, 0, st, a, per_octant);            \
        return hipGetLastError();                                                                        \
    }
    DVM_SWEEP_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

inline int sweep_config_list(int nh, int *threads, int *wpe, int cap) {
    int n = 0;
#define X(NH, K, W)                             \
    if (nh == NH) {                             \
        if (n < cap) {                          \
            threads[n] = SweepShape<NH>::T;     \
            wpe[n] = K;                         \
        }                                       \
        ++n;                                    \
    }
    DVM_SWEEP_CONFIGS(X)
#undef X
    return n;
}

inline bool sweep_config_exists(int nh, int threads, int wg_per_cu) {
#define X(NH, K, W) \
    if (nh == NH && threads == SweepShape<NH>::T && (wg_per_cu == 0 || wg_per_cu == K)) return true;
    DVM_SWEEP_CONFIGS(X)
#undef X
    return false;
}

}  // namespace impl
}  // namespace dvm
