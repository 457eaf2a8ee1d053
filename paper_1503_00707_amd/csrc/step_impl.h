// step_impl.h -- device templates of the DVM-BGK step, instantiated per
// storage precision in kernels_f32.hip / kernels_f64.hip.
//
// Layout.  f is [cell][velocity] with the velocity index innermost; the 8
// velocity sign groups ("octants") are contiguous blocks of B = NH^3 nodes,
// (-,-,-) first and the z sign fastest (section 3.1, step 1); inside an
// octant, slot s = (ax*NH + ay)*NH + az has |xi_b| = (a_b + 1/2) dv_b.  A
// workgroup owns one cell: thread t handles slots t, t+T, ... in every octant,
// so (a) the |xi| of a thread's slots are the same in all 8 octants and only
// the signs change, (b) within one octant all lanes read the same upwind
// neighbour row: the upwind choice is a compile-time function of the octant
// and the row pointer is workgroup-uniform, and 64 lanes read 256 contiguous
// bytes of it.
//
// One step per cell, fused into one pass over HBM (read f once, write f once):
//   transport   eq. (2) in flux form, f* = f - dt/h sum_b |xi_b| (f - f_up,b);
//               f_up is the upwind neighbour (SAME/COARSER), the mean of the
//               four finer neighbours (FINER: 4 sub-faces of area (h/2)^2), or
//               a ghost value (inflow Maxwellian, own value at an outflow face,
//               diffuse-wall re-emission).  Cells with only single-row faces
//               take a branch-free path whose neighbour loads are all
//               independent of each other (the compiler hoists them).
//   moments     FP64 sums w sum (1, xi, |xi|^2/2) f*: the 8 octant values of a
//               slot are combined by an FP64 Walsh butterfly, lane partials go
//               through a wave butterfly and LDS (the O(log n) tree of
//               section 3.2).
//   Maxwellian  separable: one wave per axis computes its N exponentials and
//               five 1D power sums; the 5x5 Gram system of eq. (6) in a
//               centred basis is assembled from those 15 sums and solved in
//               FP64 by every thread (no further barrier).
//   relaxation  f' = e f* + (1-e) Mt, Mt = C g_x g_y g_z (P_x + P_y + P_z).
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

#include "kernels.h"

namespace dvm {
namespace impl {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Read-only data with a workgroup-uniform address, read through the constant
// address space so that the loads are scalar (they do not count against the
// vector-memory counter of the data loads in flight).
typedef __attribute__((address_space(4))) const uint32_t cuint32_t;
template <typename F>
using cF = __attribute__((address_space(4))) const F;
template <typename T>
__device__ __forceinline__ cF<T> *as_const_space(const T *p) {
    return (cF<T> *)p;  // generic -> constant address space (a C cast: no C++ cast crosses spaces)
}

// A double moved across lanes by a DPP pattern (both 32-bit halves); the
// patterns used here take every source lane from the same row of 16.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = uint32_t(__builtin_amdgcn_mov_dpp(int(uint32_t(u)), CTRL, 0xf, 0xf, false));
    const uint32_t hi = uint32_t(__builtin_amdgcn_mov_dpp(int(uint32_t(u >> 32)), CTRL, 0xf, 0xf, false));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u)), lane));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u >> 32)), lane));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// A double read from another lane of the wave (any index; taken modulo 64).
__device__ __forceinline__ double shfl_f64(double v, int src) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int addr = (src & 63) << 2;
    const uint32_t lo = uint32_t(__builtin_amdgcn_ds_bpermute(addr, int(uint32_t(u))));
    const uint32_t hi = uint32_t(__builtin_amdgcn_ds_bpermute(addr, int(uint32_t(u >> 32))));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// Sum over the 64 lanes of a wave (every lane active); every lane receives
// the same total.  Within a row of 16 lanes: pairs (lane ^ 1), pairs of
// pairs (lane ^ 2), then the mirrored half-row and the mirrored row, each a
// commutative exchange, so all 16 lanes hold the identical row sum; the four
// row sums are then read as uniform values and added in a fixed order.
__device__ inline double wave_sum(double v) {
    v += dpp_f64<0xb1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4e>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Sum K values over the workgroup; every thread receives the same totals in
// a fixed combination order (deterministic).
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
// runs of 2^lg consecutive cells (a bijection on [0, nb); the tail that does
// not fill a whole round keeps the identity).  Scalar: the result is uniform.
__device__ inline uint32_t remap_cell(uint32_t b, uint32_t nb, int lg) {
    const uint32_t chunk = 8u << lg;
    const uint32_t full = nb - (nb & (chunk - 1));
    uint32_t c = b;
    if (b < full) {
        const uint32_t xcd = b & 7u, local = b >> 3;
        c = ((local >> lg) << (lg + 3)) + (xcd << lg) + (local & ((1u << lg) - 1));
    }
    return __builtin_amdgcn_readfirstlane(c);
}

// Row access through raw buffer instructions: one 4-SGPR descriptor per row
// (base address, byte size), a per-lane 32-bit byte offset shared by every
// row and a scalar byte offset per octant.  Out-of-range offsets read 0 and
// drop writes instead of faulting.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // 32-bit data format, raw (untyped) access
constexpr int kAuxNT = 2;               // non-temporal cache policy

// Every row base is workgroup-uniform by construction; readfirstlane states it
// so that descriptors live in SGPRs (no per-lane waterfall around the loads).
__device__ __forceinline__ Rsrc rsrc(const void *p, uint32_t bytes) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    void *u = reinterpret_cast<void *>((uint64_t(hi) << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(u, short(0), int(bytes), kRsrcWord3);
}
// A workgroup-uniform value read by every lane (from LDS, say), moved to
// scalar registers.
__device__ __forceinline__ float uniform_value(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, x)));
}
__device__ __forceinline__ double uniform_value(double x) {
    const uint64_t v = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

template <typename F>
__device__ __forceinline__ F bld(Rsrc r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float bld<float>(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
}
template <>
__device__ __forceinline__ double bld<double>(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0));
}
template <typename F, int AUX>
__device__ __forceinline__ void bst(Rsrc r, uint32_t voff, uint32_t soff, F v);
template <>
__device__ __forceinline__ void bst<float, 0>(Rsrc r, uint32_t voff, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(voff), int(soff), 0);
}
template <>
__device__ __forceinline__ void bst<float, kAuxNT>(Rsrc r, uint32_t voff, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(voff), int(soff), kAuxNT);
}
template <>
__device__ __forceinline__ void bst<double, 0>(Rsrc r, uint32_t voff, uint32_t soff, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          int(voff), int(soff), 0);
}
template <>
__device__ __forceinline__ void bst<double, kAuxNT>(Rsrc r, uint32_t voff, uint32_t soff, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          int(voff), int(soff), kAuxNT);
}

// The 128-byte cell record, read once as dwords at kernel entry (uniform
// scalar loads): words 0..23 the neighbour table, word 24 the kinds of faces
// 0..3, word 25 the kinds of faces 4..5, the level and the flags.
struct CellView {
    uint32_t w[26];
    const uint32_t *p;
    __device__ __forceinline__ CellView(const DevCell *cells, int64_t c)
        : p(reinterpret_cast<const uint32_t *>(cells + c)) {
#pragma unroll
        for (int k = 0; k < 26; ++k) w[k] = __builtin_amdgcn_readfirstlane(p[k]);
    }
    // runtime-indexed reads go to memory (scalar loads), not to a register array
    __device__ __forceinline__ int type_rt(int f) const {
        return (__builtin_amdgcn_readfirstlane(p[24 + (f >> 2)]) >> (8 * (f & 3))) & 0xff;
    }
    __device__ __forceinline__ int32_t nbr_rt(int f, int k) const {
        return int32_t(__builtin_amdgcn_readfirstlane(p[4 * f + k]));
    }
    __device__ __forceinline__ int type(int f) const {
        return f < 4 ? (w[24] >> (8 * f)) & 0xff : (w[25] >> (8 * (f - 4))) & 0xff;
    }
    __device__ __forceinline__ int level() const { return (w[25] >> 16) & 0xff; }
    __device__ __forceinline__ int flags() const { return w[25] >> 24; }
    __device__ __forceinline__ int32_t nbr(int f, int k) const { return int32_t(w[4 * f + k]); }
};

template <int NH>
__device__ inline void slot_axes(int s, int &ax, int &ay, int &az) {
    ax = s / (NH * NH);
    ay = (s / NH) % NH;
    az = s % NH;
}

// Thread -> velocity-slot map: thread t owns slots t + q*T, q < S, in every
// octant, so one vector offset t*sizeof(F) addresses every row and the round
// and octant offsets are scalar constants.  When T is a multiple of NH^2 the
// thread's ay, az (hence |xi_y|, |xi_z|) are the same in every round and only
// ax = t / NH^2 + q * T / NH^2 changes; otherwise the axes are decoded per
// round.  Slots s >= B (padding of the last round) are not stored.
template <int NH, int T>
struct Lane {
    static constexpr int B = NH * NH * NH;
    static constexpr int S = (B + T - 1) / T;
    static constexpr bool kQInv = S == 1 || T % (NH * NH) == 0;
    __device__ __forceinline__ int slot(int q) const { return int(threadIdx.x) + q * T; }
    __device__ __forceinline__ bool ok(int q) const { return S * T == B || slot(q) < B; }
    __device__ __forceinline__ void axes(int q, int &ax, int &ay, int &az) const {
        if (kQInv) {
            const int t = threadIdx.x;
            az = t % NH;
            ay = (t / NH) % NH;
            ax = t / (NH * NH) + q * (T / (NH * NH));
        } else {
            slot_axes<NH>(slot(q), ax, ay, az);
        }
    }
    // the same decode from a copy of the thread index the optimizer cannot
    // see through: used late in a step, so that the early decode is not kept
    // alive (in registers or spilled) across the whole step
    __device__ __forceinline__ void axes_late(int q, int &ax, int &ay, int &az) const {
        int t = int(threadIdx.x);
        asm volatile("" : "+v"(t));
        if (kQInv) {
            az = t % NH;
            ay = (t / NH) % NH;
            ax = t / (NH * NH) + q * (T / (NH * NH));
        } else {
            slot_axes<NH>(t + q * T, ax, ay, az);
        }
    }
    template <typename F>
    static constexpr uint32_t soff(int o, int q) {
        return uint32_t((o * B + q * T) * sizeof(F));
    }
};

// The state values a thread keeps in registers during a step: [octant][round].
template <typename F, int NH, int T>
using Regs = F[8][Lane<NH, T>::S];

template <typename F, int NH>
struct MaxwellSmem {
    static constexpr int N = 2 * NH;
    double S[15];
    double d[5];
    double C;
    double g[3][N];
    double c[3][N];
    F tab[3][N][2];  // (G, P) per axis and node
};

// Entry (i, j) of the Gram matrix G'_ij = sum_i phi_i phi_j g_x g_y g_z dv^3
// in the basis phi = (1, cx, cy, cz, |c|^2), from the 1D sums X, Y, Z (power
// p of c at index p).
__device__ inline double gram_entry(int i, int j, const double *X, const double *Y, const double *Z) {
    const int ex = (i == 1) + (j == 1), ey = (i == 2) + (j == 2), ez = (i == 3) + (j == 3);
    const int n4 = (i == 4) + (j == 4);
    if (n4 == 0) return X[ex] * Y[ey] * Z[ez];
    if (n4 == 1) return X[ex + 2] * Y[ey] * Z[ez] + X[ex] * Y[ey + 2] * Z[ez] + X[ex] * Y[ey] * Z[ez + 2];
    return X[4] * Y[0] * Z[0] + X[0] * Y[4] * Z[0] + X[0] * Y[0] * Z[4] +
           2.0 * (X[2] * Y[2] * Z[0] + X[2] * Y[0] * Z[2] + X[0] * Y[2] * Z[2]);
}

// Corrected discrete Maxwellian of (rho, u, T) as separable tables:
//   Mt_i = C g_x g_y g_z (1 + d.phi_i),  phi = (1, cx, cy, cz, |c|^2),
//   c = (xi - u)/sqrt(T), g = exp(-c^2/2), C = rho (2 pi T)^(-3/2).
// d solves G d = r with G_ab = w sum_i phi_a phi_b M_i (the five conservation
// equations of eq. 6 in a centred basis spanning the same polynomials) and
// r = (rho, 0, 0, 0, 3 rho) - G[:,0], the phi-moments of the target minus
// those of the raw Maxwellian.  Every entry of G is a product of 1D sums
// S_b,p = dv_b sum_k c_k^p g_k, so the cost per cell is O(N), not O(N^3).
// The 5x6 augmented system is eliminated Gauss-Jordan style by 30 lanes of
// the first wave, one element per lane in a register (G is symmetric
// positive definite, so no pivoting).  tab[0] carries C * mfac, so that the table
// product is mfac * Mt.
template <typename F, int NH, int T>
__device__ __forceinline__ void maxwell_solve(MaxwellSmem<F, NH> &sm, double rho, const double u[3], double Tt,
                                              const VelGrid &g) {
    constexpr int N = 2 * NH;
    constexpr int NW = (T + 63) / 64;
    static_assert(N <= 64, "one wave per axis");
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int b = wid; b < 3; b += NW) {
        double gk = 0.0, ck = 0.0;
        if (lane < N) {
            const double xi = (double(lane - NH) + 0.5) * g.dv[b];
            ck = (xi - u[b]) / sqrt(Tt);
            gk = exp(-0.5 * ck * ck);
            sm.g[b][lane] = gk;
            sm.c[b][lane] = ck;
        }
        double p[5];
        p[0] = gk;
#pragma unroll
        for (int q = 1; q < 5; ++q) p[q] = p[q - 1] * ck;
#pragma unroll
        for (int q = 0; q < 5; ++q) p[q] = wave_sum(p[q]);
        if (lane == 0)
            for (int q = 0; q < 5; ++q) sm.S[5 * b + q] = p[q] * g.dv[b];
    }
    __syncthreads();
    if (wid == 0) {
        const int i = lane / 6, j = lane % 6;
        const bool el = lane < 30;
        const double x2 = 6.283185307179586476925286766559 * Tt;
        const double C = rho / (x2 * sqrt(x2));
        // lane 6i + j holds A[i][j]; each elimination step reads the pivot
        // row and column from the lanes that hold them (no LDS round trip)
        double x = 0.0;
        if (el) {
            if (j < 5) x = gram_entry(i, j, &sm.S[0], &sm.S[5], &sm.S[10]);
            else {
                const double t = (i == 0 ? 1.0 : i == 4 ? 3.0 : 0.0) * (rho / C);
                x = t - gram_entry(i, 0, &sm.S[0], &sm.S[5], &sm.S[10]);
            }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const double akk = readlane_f64(x, 7 * k);
            const double aik = shfl_f64(x, 6 * i + k);
            const double akj = shfl_f64(x, 6 * k + j);
            if (el && i != k) x = x - aik / akk * akj;
        }
        const double diag = shfl_f64(x, 7 * lane), rhs = shfl_f64(x, 6 * lane + 5);
        if (lane < 5) sm.d[lane] = rhs / diag;
        if (lane == 0) sm.C = C;
    }
    __syncthreads();
}

// Fill the storage-precision tables from a solved Maxwellian (after
// maxwell_solve): tab[0] carries C * mfac, so the table product is mfac * Mt.
template <typename F, int NH, int T>
__device__ void maxwell_fill(MaxwellSmem<F, NH> &sm, double mfac) {
    constexpr int N = 2 * NH;
    constexpr int NW = (T + 63) / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int b = wid; b < 3; b += NW) {
        if (lane < N) {
            const double cc = sm.c[b][lane];
            const double P = b == 0 ? 1.0 + sm.d[0] + sm.d[1] * cc + sm.d[4] * cc * cc
                                    : sm.d[1 + b] * cc + sm.d[4] * cc * cc;
            const double G = b == 0 ? sm.g[b][lane] * sm.C * mfac : sm.g[b][lane];
            sm.tab[b][lane][0] = F(G);
            sm.tab[b][lane][1] = F(P);
        }
    }
    __syncthreads();
}

template <typename F, int NH, int T>
__device__ __forceinline__ void maxwell_tables(MaxwellSmem<F, NH> &sm, double rho, const double u[3], double Tt,
                                               double mfac, const VelGrid &g) {
    maxwell_solve<F, NH, T>(sm, rho, u, Tt, g);
    maxwell_fill<F, NH, T>(sm, mfac);
}

// Write f' = e*fs + M' for the slots of this thread, M' from the tables.
template <typename F, int NH, int T, bool NT>
__device__ inline void relax_store(const MaxwellSmem<F, NH> &sm, const Regs<F, NH, T> &fo, F e, Rsrc out) {
    using L = Lane<NH, T>;
    const L ln;
    const uint32_t voff = threadIdx.x * sizeof(F);
#pragma unroll
    for (int q = 0; q < L::S; ++q) {
        if (!ln.ok(q)) continue;
        int a3[3];
        ln.axes_late(q, a3[0], a3[1], a3[2]);  // recomputed: nothing held across the step for it
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
            const F M = (G[0][ox] * G[1][oy]) * G[2][oz] * ((P[0][ox] + P[1][oy]) + P[2][oz]);
            bst<F, NT ? kAuxNT : 0>(out, voff, L::template soff<F>(o, q), e * fo[o][q] + M);
        }
    }
}

// FP64 Walsh butterfly over the 8 octant values of one slot:
// s0 = sum, sx/sy/sz = signed sums along each axis (o = ox*4 + oy*2 + oz).
template <typename F, int S>
__device__ inline void octant_sums(const F (&v)[8][S], int q, double &s0, double &sx, double &sy, double &sz) {
    double d[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) d[o] = double(v[o][q]);
    const double p0 = d[4] + d[0], m0 = d[4] - d[0];
    const double p1 = d[5] + d[1], m1 = d[5] - d[1];
    const double p2 = d[6] + d[2], m2 = d[6] - d[2];
    const double p3 = d[7] + d[3], m3 = d[7] - d[3];
    sx = (m0 + m1) + (m2 + m3);
    const double q0 = p2 + p0, n0 = p2 - p0;
    const double q1 = p3 + p1, n1 = p3 - p1;
    sy = n0 + n1;
    s0 = q1 + q0;
    sz = q1 - q0;
}

// Per-thread FP64 partial sums (1, xi, |xi|^2/2) f over the thread's slots.
template <typename F, int NH, int T>
__device__ __forceinline__ void add_moments(const Regs<F, NH, T> &fo, const VelGrid &g, double (&m)[5]) {
    using L = Lane<NH, T>;
    constexpr int S = L::S;
    const L ln;
#pragma unroll
    for (int q = 0; q < S; ++q) {
        if (!ln.ok(q)) continue;
        int a3[3];
        ln.axes_late(q, a3[0], a3[1], a3[2]);
        const double xa = (a3[0] + 0.5) * g.dv[0];
        const double ya = (a3[1] + 0.5) * g.dv[1];
        const double za = (a3[2] + 0.5) * g.dv[2];
        double s0, sx, sy, sz;
        octant_sums<F, S>(fo, q, s0, sx, sy, sz);
        m[0] += s0;
        m[1] += xa * sx;
        m[2] += ya * sy;
        m[3] += za * sz;
        m[4] += 0.5 * (xa * xa + ya * ya + za * za) * s0;
    }
}

template <typename F, int NH, int T>
struct StepSmem {
    static constexpr int NW = (T + 63) / 64;
    double red[NW * 5];
    double rho_w[6];
    MaxwellSmem<F, NH> mx;
    // FP32: landing area of the FINER / WALL correction loads (per wave: 4
    // rows x S rounds x 64 lanes), filled by loads that write LDS directly
    float stage[std::is_same<F, float>::value ? NW : 1][std::is_same<F, float>::value ? 4 * Lane<NH, T>::S : 1][64];
};

// Transport of the thread's slots; fo holds f on entry and f* on return.
// Main pass: per octant the three upwind faces are compile-time constants and
// every face is read through one row descriptor, so the loop has no branch
// and its loads are independent (the compiler pipelines them).  FINER and
// WALL faces are given an empty descriptor there (reads return 0); the
// correction pass then adds nu * f_up for them, f_up the mean of the four
// finer rows or rho_w times the wall Maxwellian.
template <typename F, int NH, int T, bool OCT_FENCE, bool REG, bool LATE_OWN>
__device__ __forceinline__ void transport(Regs<F, NH, T> &fo, const CellView &cell, const Rsrc (&R1)[6],
                                          const Rsrc &own, const F *fin, const StepArgs &a, const double *rho_w,
                                          double dth, double (&m)[5], float *stage) {
    using L = Lane<NH, T>;
    constexpr int S = L::S;
    constexpr int64_t NV = 8 * L::B;
    constexpr uint32_t kRow = uint32_t(NV * sizeof(F));
    const L ln;
    const uint32_t voff = threadIdx.x * sizeof(F);
    F nu[3][S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        int a3[3];
        ln.axes(q, a3[0], a3[1], a3[2]);
#pragma unroll
        for (int b = 0; b < 3; ++b) nu[b][q] = F(dth) * (F(a3[b]) + F(0.5)) * F(a.g.dv[b]);
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        // a positive component enters through the low face, a negative one through the high face
        const int fx = 0 + ((o >> 2) ? 0 : 1), fy = 2 + (((o >> 1) & 1) ? 0 : 1), fz = 4 + ((o & 1) ? 0 : 1);
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const uint32_t so = L::template soff<F>(o, q);
            if constexpr (LATE_OWN) fo[o][q] = bld<F>(own, voff, so);
            const F v = fo[o][q];
            const F ux = bld<F>(R1[fx], voff, so);
            const F uy = bld<F>(R1[fy], voff, so);
            const F uz = bld<F>(R1[fz], voff, so);
            fo[o][q] = v - (nu[0][q] * (v - ux) + nu[1][q] * (v - uy) + nu[2][q] * (v - uz));
        }
        // bound the look-ahead of the scheduler to one octant: hoisting loads
        // further only trades them for spills
        if (OCT_FENCE) asm volatile("" ::: "memory");
    }
    // correction for FINER and WALL faces: a runtime loop over the faces (one
    // face's loads in flight at a time), workgroup-uniform branches; absent
    // from the reduced kernel, whose cells have no such faces
#pragma nounroll
    for (int f = 0; f < (REG ? 0 : 6); ++f) {
        const int ty = cell.type_rt(f);
        if (ty != DVM_FACE_FINER && ty != DVM_FACE_WALL) continue;
        const int b = f >> 1, enter = (f & 1) ? 0 : 1;  // sign bit of the velocities entering through f
        const bool finer = ty == DVM_FACE_FINER;
        Rsrc r[4];
        F sc;
        if (finer) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t nb = cell.nbr_rt(f, k);
                r[k] = rsrc(fin + nb * NV, kRow);
            }
            sc = F(0.25);
        } else {
            r[0] = r[1] = r[2] = r[3] = rsrc(a.wall_m1, kRow);
            sc = F(rho_w[f]);
        }
        if constexpr (std::is_same<F, float>::value) {
            // every load of an octant in flight at once, landing in this
            // wave's part of LDS (no registers held): lane l of a load writes
            // word l of its 64-word slot
            float *wst = stage + (threadIdx.x >> 6) * (4 * S * 64);
            const int lane = threadIdx.x & 63;
            const int nk = finer ? 4 : 1;
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                if (((o >> (2 - b)) & 1) != enter) continue;
#pragma unroll
                for (int q = 0; q < S; ++q)
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (k < nk)
                            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                                r[k], (__attribute__((address_space(3))) void *)(wst + (q * 4 + k) * 64), 4, voff,
                                L::template soff<F>(o, q), 0, 0);
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    const float *v = wst + q * 4 * 64 + lane;
                    const F up = finer ? (v[0] + v[64]) + (v[128] + v[192]) : v[0];
                    const F nub = b == 0 ? nu[0][q] : b == 1 ? nu[1][q] : nu[2][q];
                    fo[o][q] += nub * (sc * up);
                }
                // the slots are read before the next octant's loads overwrite them
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            }
        } else {
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int sg[3] = {o >> 2, (o >> 1) & 1, o & 1};
            if (sg[b] != enter) continue;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const uint32_t so = L::template soff<F>(o, q);
                F up = bld<F>(r[0], voff, so);
                if (finer) up = (up + bld<F>(r[1], voff, so)) + (bld<F>(r[2], voff, so) + bld<F>(r[3], voff, so));
                const F nub = b == 0 ? nu[0][q] : b == 1 ? nu[1][q] : nu[2][q];
                fo[o][q] += nub * (sc * up);
            }
            asm volatile("" ::: "memory");
        }
        }
    }
    add_moments<F, NH, T>(fo, a.g, m);
}

// ---------------------------------------------------------------------------
// MUSCL-minmod transport inside the step (no face-value buffers).  The paper
// is silent on the reconstruction; the reading: per cell x, axis b and
// velocity, sigma = minmod((f - fm)/dm, (fp - f)/dp), fm and fp the low- and
// high-side face-neighbour values -- the neighbour's average (SAME, COARSER),
// the mean of the four finer leaves (FINER), the inflow ghost (INFLOW) or the
// cell's own value (OUTFLOW) -- and dm, dp the centre distances h, 3h/4
// (FINER), 3h/2 (COARSER); sigma = 0 in a cell that touches a wall.  The value
// a cell lets through the face its velocity leaves by is
//   D = f + sgn(xi_b) (h/2) sigma_b,
// the cell's own outflow on that face and its downwind neighbour's inflow.  A
// step therefore reads, per octant and axis, the cell's two face neighbours
// (its own slope) and, behind its upwind neighbour, that neighbour's far
// neighbour (the upwind slope): two hops along each axis.
// ---------------------------------------------------------------------------

template <typename F>
__device__ __forceinline__ F minmod(F l, F r) {
    return l * r <= F(0) ? F(0) : (fabs(l) < fabs(r) ? l : r);
}

// A cell record read word by word through scalar loads (a neighbour's, used
// for a few fields only).
struct RecRT {
    cuint32_t *p;
    __device__ __forceinline__ RecRT(const DevCell *cells, int64_t x)
        : p(as_const_space(reinterpret_cast<const uint32_t *>(cells + x))) {}
    __device__ __forceinline__ int type(int f) const { return (p[24 + (f >> 2)] >> (8 * (f & 3))) & 0xff; }
    __device__ __forceinline__ int32_t nbr(int f, int k) const { return int32_t(p[4 * f + k]); }
    __device__ __forceinline__ int level() const { return (p[25] >> 16) & 0xff; }
    __device__ __forceinline__ int flags() const { return p[25] >> 24; }
};

// Every face of the cell is SAME, INFLOW, OUTFLOW or WALL, and behind no SAME
// face lies a FINER face: each value its MUSCL stencil reads is one row (the
// branch-free code).
__device__ __forceinline__ bool muscl_single_row(const DevCell *cells, int64_t c) {
    const RecRT r(cells, c);
    bool ok = true;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int ty = r.type(f);
        if (ty == DVM_FACE_SAME) ok &= RecRT(cells, r.nbr(f, 0)).type(f) != DVM_FACE_FINER;
        else ok &= ty == DVM_FACE_INFLOW || ty == DVM_FACE_OUTFLOW || ty == DVM_FACE_WALL;
    }
    return ok;
}

// Value of cell x's face neighbour across face f for the thread's slots of
// octant o (mean of the rows of a FINER face), and 1 / centre distance.
// own: x's values (the OUTFLOW side).
template <typename F, int NH, int T>
__device__ __forceinline__ void muscl_side(const StepArgs &a, const RecRT &x, double h, int f, int o,
                                           const F (&own)[Lane<NH, T>::S], F (&out)[Lane<NH, T>::S], F &inv) {
    using L = Lane<NH, T>;
    constexpr int S = L::S;
    constexpr int64_t NV = 8 * L::B;
    constexpr uint32_t kRow = uint32_t(NV * sizeof(F));
    const F *fin = static_cast<const F *>(a.f_in);
    const uint32_t voff = threadIdx.x * sizeof(F);
    const int ty = x.type(f);
    if (ty == DVM_FACE_SAME || ty == DVM_FACE_COARSER || ty == DVM_FACE_INFLOW) {
        const Rsrc r = rsrc(ty == DVM_FACE_INFLOW ? static_cast<const F *>(a.ghost_in) : fin + int64_t(x.nbr(f, 0)) * NV,
                            kRow);
#pragma unroll
        for (int q = 0; q < S; ++q) out[q] = bld<F>(r, voff, L::template soff<F>(o, q));
        inv = F(1.0 / (ty == DVM_FACE_COARSER ? 1.5 * h : h));
    } else if (ty == DVM_FACE_FINER) {
        Rsrc r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = rsrc(fin + int64_t(x.nbr(f, k)) * NV, kRow);
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const uint32_t so = L::template soff<F>(o, q);
            out[q] = F(0.25) * (((bld<F>(r[0], voff, so) + bld<F>(r[1], voff, so)) + bld<F>(r[2], voff, so)) +
                                bld<F>(r[3], voff, so));
        }
        inv = F(1.0 / (0.75 * h));
    } else {  // OUTFLOW (WALL: the slope is zero anyway)
#pragma unroll
        for (int q = 0; q < S; ++q) out[q] = own[q];
        inv = F(1.0 / h);
    }
}

// D of cell x on axis b for the thread's slots of octant o, the velocity
// component's sign bit sb (1: positive, the value at x's high face).
template <typename F, int NH, int T>
__device__ __forceinline__ void muscl_face_value(const StepArgs &a, int64_t x, int b, int sb, int o,
                                                 F (&out)[Lane<NH, T>::S]) {
    using L = Lane<NH, T>;
    constexpr int S = L::S;
    constexpr int64_t NV = 8 * L::B;
    const F *fin = static_cast<const F *>(a.f_in);
    const uint32_t voff = threadIdx.x * sizeof(F);
    const RecRT r(a.cells, x);
    const Rsrc row = rsrc(fin + x * NV, uint32_t(NV * sizeof(F)));
    F fx[S];
#pragma unroll
    for (int q = 0; q < S; ++q) fx[q] = bld<F>(row, voff, L::template soff<F>(o, q));
    if (r.flags() & 1) {
#pragma unroll
        for (int q = 0; q < S; ++q) out[q] = fx[q];
        return;
    }
    const double h = a.h0 / double(1 << r.level());
    F lo[S], hi[S], ilo, ihi;
    muscl_side<F, NH, T>(a, r, h, 2 * b, o, fx, lo, ilo);
    muscl_side<F, NH, T>(a, r, h, 2 * b + 1, o, fx, hi, ihi);
    const F half = F(sb ? 0.5 * h : -0.5 * h);
#pragma unroll
    for (int q = 0; q < S; ++q) out[q] = fx[q] + half * minmod((fx[q] - lo[q]) * ilo, (hi[q] - fx[q]) * ihi);
}

// MUSCL transport of the thread's slots; fo holds f on entry (FAST with
// LATE_OWN: loaded here, octant by octant) and f* on return.
//   FAST: the cells of muscl_single_row: per face the neighbour row and the
//         row behind the neighbour, selected once per cell; the loads of an
//         octant are independent of each other and issued together;
//         WALLS: such a cell with a diffuse-wall face (no slope of its own;
//         through a wall face enters rho_w times the wall Maxwellian), whose
//         wall densities are in rho_w;
//   else: any cell (level jumps on either hop, walls): the stencil is read
//         from the neighbours' records, axis by axis.
template <typename F, int NH, int T, bool FAST, bool LATE_OWN, bool WALLS = false>
__device__ __forceinline__ void transport_muscl(Regs<F, NH, T> &fo, const CellView &cell, int64_t c,
                                                const Rsrc &own, const StepArgs &a, const double *rho_w, double dth,
                                                double (&m)[5]) {
    using L = Lane<NH, T>;
    constexpr int S = L::S;
    constexpr int64_t NV = 8 * L::B;
    constexpr uint32_t kRow = uint32_t(NV * sizeof(F));
    const L ln;
    const uint32_t voff = threadIdx.x * sizeof(F);
    const F *fin = static_cast<const F *>(a.f_in);
    const double h = a.h0 / double(1 << cell.level());
    const F hh = F(0.5 * h), ih = F(1.0 / h);
    if constexpr (FAST) {
        // per face f: the cell whose row lies across f (the inflow ghost: -1;
        // the wall Maxwellian: -2; an OUTFLOW face: the cell itself) and,
        // behind a SAME neighbour u,
        // the next one along the axis (u itself at an OUTFLOW or WALL face);
        // 1/distance from u to that one; whether u has a slope (SAME and not
        // touching a wall)
        int32_t Ni[6], Fi[6];
        uint32_t on = 0, farc = 0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int ty = cell.type(f);
            Ni[f] = ty == DVM_FACE_SAME     ? cell.nbr(f, 0)
                    : ty == DVM_FACE_INFLOW ? -1
                    : ty == DVM_FACE_WALL   ? -2
                                            : int32_t(c);
            Fi[f] = Ni[f];
            if (ty == DVM_FACE_SAME) {
                const RecRT u(a.cells, Ni[f]);
                const int tu = u.type(f);
                if (tu == DVM_FACE_SAME || tu == DVM_FACE_COARSER) Fi[f] = u.nbr(f, 0);
                else if (tu == DVM_FACE_INFLOW) Fi[f] = -1;
                on |= uint32_t(!(u.flags() & 1)) << f;
                farc |= uint32_t(tu == DVM_FACE_COARSER) << f;
            }
        }
        // descriptors and per-face factors made once, before the octant loop
        // and without branches: a select inside the loop becomes a branch,
        // and the compiler then hoists every octant's loads and spills them
        const uint64_t ghost = reinterpret_cast<uint64_t>(a.ghost_in), base = reinterpret_cast<uint64_t>(fin);
        const uint64_t wallm = reinterpret_cast<uint64_t>(a.wall_m1);
        const auto row = [&](int32_t i) {
            const uint64_t at = base + uint64_t(int64_t(i < 0 ? 0 : i) * NV * int64_t(sizeof(F)));
            return rsrc(reinterpret_cast<const void *>(i < 0 ? (i == -1 ? ghost : wallm) : at), kRow);
        };
        const F i15 = F(1.0 / (1.5 * h));
        Rsrc RN[6], RF[6];
        F ifar[6], son[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            RN[f] = row(Ni[f]);
            RF[f] = row(Fi[f]);
            ifar[f] = (farc >> f) & 1u ? i15 : ih;
            son[f] = (on >> f) & 1u ? F(1) : F(0);
        }
        if constexpr (WALLS) {
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int sg[3] = {o >> 2, (o >> 1) & 1, o & 1};
                // rho_w on a wall face, 1 on the others (an exact product);
                // read per octant, after the fence, to keep them out of the
                // registers the loads need
                F sN[3];
#pragma unroll
                for (int b = 0; b < 3; ++b) sN[b] = uniform_value(F(rho_w[sg[b] ? 2 * b : 2 * b + 1]));
                F up[3][S], far[3][S];
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    const uint32_t so = L::template soff<F>(o, q);
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const int fu = sg[b] ? 2 * b : 2 * b + 1;
                        up[b][q] = bld<F>(RN[fu], voff, so);
                        far[b][q] = bld<F>(RF[fu], voff, so);
                    }
                }
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    int a3[3];
                    ln.axes_late(q, a3[0], a3[1], a3[2]);
                    const F v = fo[o][q];
                    F t = F(0);
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const int fu = sg[b] ? 2 * b : 2 * b + 1;
                        const F half = sg[b] ? hh : -hh;
                        // son is 0 on a wall face: there the slope drops out
                        // and din is rho_w times the wall row
                        const F u = up[b][q];
                        const F su = sg[b] ? minmod((u - far[b][q]) * ifar[fu], (v - u) * ih)
                                           : minmod((u - v) * ih, (far[b][q] - u) * ifar[fu]);
                        const F din = sN[b] * u + half * (son[fu] * su);
                        const F nub = F(dth) * (F(a3[b]) + F(0.5)) * F(a.g.dv[b]);
                        t += nub * (v - din);  // a wall cell has no slope of its own
                    }
                    fo[o][q] = v - t;
                }
                asm volatile("" ::: "memory");  // one octant's loads in flight at a time
            }
        } else {
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int sg[3] = {o >> 2, (o >> 1) & 1, o & 1};
            F lo[3][S], hi[3][S], far[3][S];
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const uint32_t so = L::template soff<F>(o, q);
                if constexpr (LATE_OWN) fo[o][q] = bld<F>(own, voff, so);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    lo[b][q] = bld<F>(RN[2 * b], voff, so);
                    hi[b][q] = bld<F>(RN[2 * b + 1], voff, so);
                    far[b][q] = bld<F>(RF[sg[b] ? 2 * b : 2 * b + 1], voff, so);  // a positive component enters through the low face
                }
            }
#pragma unroll
            for (int q = 0; q < S; ++q) {
                int a3[3];
                ln.axes_late(q, a3[0], a3[1], a3[2]);
                const F v = fo[o][q];
                F t = F(0);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const int fu = sg[b] ? 2 * b : 2 * b + 1;
                    const F half = sg[b] ? hh : -hh;
                    const F dc = v + half * minmod((v - lo[b][q]) * ih, (hi[b][q] - v) * ih);
                    const F up = sg[b] ? lo[b][q] : hi[b][q];
                    const F su = sg[b] ? minmod((up - far[b][q]) * ifar[fu], (v - up) * ih)
                                       : minmod((up - v) * ih, (far[b][q] - up) * ifar[fu]);
                    const F din = up + half * (son[fu] * su);
                    const F nub = F(dth) * (F(a3[b]) + F(0.5)) * F(a.g.dv[b]);
                    t += nub * (dc - din);
                }
                fo[o][q] = v - t;
            }
            asm volatile("" ::: "memory");  // one octant's loads in flight at a time
        }
        }
    } else {
        // runtime loops over octants and axes (one copy of the code); the
        // register arrays are reached through uniform selects, never indexed
        const RecRT rc(a.cells, c);
        const bool wall = cell.flags() & 1;
#pragma nounroll
        for (int o = 0; o < 8; ++o) {
            F v[S], t[S];
#pragma unroll
            for (int q = 0; q < S; ++q) {
                v[q] = fo[0][q];
#pragma unroll
                for (int k = 1; k < 8; ++k) v[q] = o == k ? fo[k][q] : v[q];
                t[q] = F(0);
            }
#pragma nounroll
            for (int b = 0; b < 3; ++b) {
                const int sb = (o >> (2 - b)) & 1;
                const F half = sb ? hh : -hh;
                F dc[S], in[S];
                if (wall) {
#pragma unroll
                    for (int q = 0; q < S; ++q) dc[q] = v[q];
                } else {
                    F lo[S], hi[S], ilo, ihi;
                    muscl_side<F, NH, T>(a, rc, h, 2 * b, o, v, lo, ilo);
                    muscl_side<F, NH, T>(a, rc, h, 2 * b + 1, o, v, hi, ihi);
#pragma unroll
                    for (int q = 0; q < S; ++q) dc[q] = v[q] + half * minmod((v[q] - lo[q]) * ilo, (hi[q] - v[q]) * ihi);
                }
                const int fu = sb ? 2 * b : 2 * b + 1;  // a positive component enters through the low face
                const int ty = rc.type(fu);
                if (ty == DVM_FACE_SAME || ty == DVM_FACE_COARSER || ty == DVM_FACE_FINER) {
                    // one upwind cell, or four behind sub-faces of a quarter of the area each
                    const int nk = ty == DVM_FACE_FINER ? 4 : 1;
#pragma nounroll
                    for (int k = 0; k < nk; ++k) {
                        F x[S];
                        muscl_face_value<F, NH, T>(a, rc.nbr(fu, k), b, sb, o, x);
#pragma unroll
                        for (int q = 0; q < S; ++q) in[q] = k == 0 ? x[q] : in[q] + x[q];
                    }
                    if (nk == 4) {
#pragma unroll
                        for (int q = 0; q < S; ++q) in[q] *= F(0.25);
                    }
                } else if (ty == DVM_FACE_INFLOW || ty == DVM_FACE_WALL) {
                    const bool inflow = ty == DVM_FACE_INFLOW;
                    const Rsrc r = rsrc(inflow ? a.ghost_in : a.wall_m1, kRow);
                    const F sc = inflow ? F(1) : F(rho_w[fu]);
#pragma unroll
                    for (int q = 0; q < S; ++q) in[q] = sc * bld<F>(r, voff, L::template soff<F>(o, q));
                } else {  // OUTFLOW: zero gradient
#pragma unroll
                    for (int q = 0; q < S; ++q) in[q] = v[q];
                }
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    int a3[3];
                    ln.axes_late(q, a3[0], a3[1], a3[2]);
                    const int ab = b == 0 ? a3[0] : b == 1 ? a3[1] : a3[2];
                    const double dvb = b == 0 ? a.g.dv[0] : b == 1 ? a.g.dv[1] : a.g.dv[2];
                    const F nub = F(dth) * (F(ab) + F(0.5)) * F(dvb);
                    t[q] += nub * (dc[q] - in[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const F r = v[q] - t[q];
#pragma unroll
                for (int k = 0; k < 8; ++k) fo[k][q] = o == k ? r : fo[k][q];
            }
        }
    }
    add_moments<F, NH, T>(fo, a.g, m);
}

// A step-cell hook runs after the cell's own values are loaded and before
// the transport overwrites them (the hybrid step records interface fluxes).
struct NoHook {
    template <typename F, int NH, int T>
    __device__ __forceinline__ void apply(const StepArgs &, const CellView &, int64_t, const Regs<F, NH, T> &,
                                          double *) const {}
};

// One fused step of cell c by the calling workgroup.
// MU: 0 first order, 1 MUSCL (any cell), 2 MUSCL (a cell of muscl_single_row).
template <typename F, int NH, int T, int FENCE, bool NT, int MU, bool REG = false, class Hook = NoHook>
__device__ __forceinline__ void step_cell(const StepArgs &a, int64_t c, StepSmem<F, NH, T> &sm,
                                          const Hook &hook = Hook()) {
    constexpr int B = NH * NH * NH;
    constexpr int64_t NV = 8 * B;
    using L = Lane<NH, T>;
    constexpr int S = L::S;

    const int tid = threadIdx.x;
    const L ln;
    const CellView cell(a.cells, c);
    const F *fin = static_cast<const F *>(a.f_in);
    constexpr uint32_t kRow = uint32_t(NV * sizeof(F));
    const Rsrc own = rsrc(fin + c * NV, kRow);
    const double dth = a.dt / (a.h0 / double(1 << cell.level()));

    // own values of every slot and octant, kept in registers for the step.
    // Reduced path: loaded octant by octant inside the transport pass, with
    // the upwind neighbours' values of the same octant, so that a cell's block
    // is read by the cell and by its concurrently running neighbours at about
    // the same time (it is still in L2 when they ask for it).  Full path:
    // loaded here (the wall densities and the step hook need every value
    // before the transport).
    constexpr bool kLateOwn = REG && std::is_same<Hook, NoHook>::value;
    F fo[8][S];
    const uint32_t voff = tid * sizeof(F);
    if constexpr (!kLateOwn) {
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int o = 0; o < 8; ++o) fo[o][q] = bld<F>(own, voff, L::template soff<F>(o, q));
    }

    // the MUSCL wall-cell path scales the row across every face: 1 where no
    // wall is (the wall faces' densities follow, after barriers)
    if constexpr (MU == 2 && !REG) {
        if (tid < 6) sm.rho_w[tid] = 1.0;
    }
    // diffuse walls: density of the re-emitted Maxwellian (zero net mass flux)
    if (!REG && (cell.flags() & 1)) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (cell.type(f) != DVM_FACE_WALL) continue;
            const int axis = f >> 1, side = f & 1;
            double v[1] = {0.0};
#pragma unroll
            for (int q = 0; q < S; ++q) {
                if (!ln.ok(q)) continue;
                int a3[3];
                ln.axes(q, a3[0], a3[1], a3[2]);
                const double xa = (a3[axis] + 0.5) * a.g.dv[axis];
                // the four octants leaving through this face share |xi_axis|:
                // summed in the storage precision, then widened once
                F s4 = F(0);
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const int sb = axis == 0 ? (o >> 2) : axis == 1 ? ((o >> 1) & 1) : (o & 1);
                    if (sb == side) s4 += fo[o][q];
                }
                v[0] += xa * double(s4);
            }
            block_sum<T, 1>(v, sm.red);
            if (tid == 0) sm.rho_w[f] = v[0] / a.wall_den[f];
        }
        __syncthreads();
    }

    hook.template apply<F, NH, T>(a, cell, c, fo, sm.red);

    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (MU) {
        transport_muscl<F, NH, T, MU == 2, kLateOwn, MU == 2 && !REG>(fo, cell, c, own, a, sm.rho_w, dth, m);
    } else {
        // one row descriptor per face for the main transport pass: the upwind
        // cell's average
        Rsrc R1[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int ty = cell.type(f);
            const F *row = fin + c * NV;  // OUTFLOW: zero gradient
            uint32_t bytes = kRow;
            if (ty == DVM_FACE_SAME || ty == DVM_FACE_COARSER) {
                row = fin + int64_t(cell.nbr(f, 0)) * NV;
            } else if (ty == DVM_FACE_INFLOW) {
                row = static_cast<const F *>(a.ghost_in);
            } else if (ty == DVM_FACE_FINER || ty == DVM_FACE_WALL) {
                bytes = 0;  // added by the correction pass
            }
            R1[f] = rsrc(row, bytes);
        }
        transport<F, NH, T, (FENCE != 0), REG, kLateOwn>(fo, cell, R1, own, fin, a, sm.rho_w, dth, m,
                                                         &sm.stage[0][0][0]);
    }
    block_sum<T, 5>(m, sm.red);

    const double w = a.g.w;
    const double rho = w * m[0];
    const double u[3] = {w * m[1] / rho, w * m[2] / rho, w * m[3] / rho};
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
    const Rsrc out = rsrc(static_cast<F *>(a.f_out) + c * NV, kRow);
    if (bad || a.collision == DVM_COLL_OFF) {
#pragma unroll
        for (int q = 0; q < S; ++q) {
            if (!ln.ok(q)) continue;
#pragma unroll
            for (int o = 0; o < 8; ++o) bst<F, 0>(out, voff, L::template soff<F>(o, q), fo[o][q]);
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
    maxwell_tables<F, NH, T>(sm.mx, rho, u, Tt, mfac, a.g);
    relax_store<F, NH, T, NT>(sm.mx, fo, F(e), out);
}

// The cell has a FINER or a WALL face (it needs the correction pass).
__device__ __forceinline__ bool needs_correction(const DevCell *cells, int64_t c) {
    cuint32_t *rec = as_const_space(reinterpret_cast<const uint32_t *>(cells + c));
    const uint32_t k0 = rec[24], k1 = rec[25];
    bool r = false;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const uint32_t ty = ((f < 4 ? k0 : k1) >> (8 * (f & 3))) & 0xffu;
        r |= ty == DVM_FACE_FINER || ty == DVM_FACE_WALL;
    }
    return r;
}

// One fused step, one cell per workgroup: every cell, or the cells listed in
// a.sel (REG: a list of cells without FINER or WALL faces).  MU: MUSCL, the
// branch-free code for the cells whose stencil values are single rows, the
// general code for the others (uniform branch).
template <typename F, int NH, int T, int WPE, int FENCE, bool NT, bool MU = false, bool REG = false>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_step(StepArgs a) {
    static_assert(T % 64 == 0, "whole waves: the wave sums read every lane");
    __shared__ StepSmem<F, NH, T> sm;
    const uint32_t b = remap_cell(blockIdx.x, gridDim.x, a.xcd_log2);
    const int64_t c = a.sel ? int64_t(as_const_space(a.sel)[b]) : int64_t(b);
    if constexpr (MU) {
        if (!muscl_single_row(a.cells, c)) step_cell<F, NH, T, FENCE, NT, 1, false>(a, c, sm);
        else if (RecRT(a.cells, c).flags() & 1) step_cell<F, NH, T, FENCE, NT, 2, false>(a, c, sm);
        else step_cell<F, NH, T, FENCE, NT, 2, true>(a, c, sm);
    } else if constexpr (!REG) {
        // every cell in one launch: the reduced code for the cells without
        // FINER or WALL faces, the full code for the others (uniform branch)
        if (needs_correction(a.cells, c)) step_cell<F, NH, T, FENCE, NT, false, false>(a, c, sm);
        else step_cell<F, NH, T, FENCE, NT, false, true>(a, c, sm);
    } else {
        step_cell<F, NH, T, FENCE, NT, false, true>(a, c, sm);
    }
}

// Batched step: the cells of many independent instances with the same
// velocity grid size in one launch.  Workgroups [wg_end[i-1], wg_end[i]) serve
// instance i (instances listed by decreasing cost, so that the largest start
// first); each reads its instance's arguments with scalar loads.
template <typename F, int NH, int T, int WPE, int FENCE, bool NT>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_step_batch(
    const StepArgs *__restrict__ inst, const uint32_t *__restrict__ wg_end, int n_inst, int xcd_log2) {
    __shared__ StepSmem<F, NH, T> sm;
    const uint32_t b = remap_cell(blockIdx.x, gridDim.x, xcd_log2);
    cuint32_t *we = as_const_space(wg_end);
    int lo = 0, hi = n_inst - 1;  // first i with wg_end[i] > b
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (we[mid] > b) hi = mid;
        else lo = mid + 1;
    }
    const uint32_t start = lo == 0 ? 0u : we[lo - 1];
    // the instance's arguments read in place (uniform address: scalar loads;
    // a private copy would live in scratch memory, an LDS copy costs an LDS
    // read at every use)
    const StepArgs &a = inst[lo];
    const int64_t c = int64_t(b - start);
    if (needs_correction(a.cells, c)) step_cell<F, NH, T, FENCE, NT, false, false>(a, c, sm);
    else step_cell<F, NH, T, FENCE, NT, false, true>(a, c, sm);
}

// f := corrected Maxwellian of a prescribed state (init and ghost rows).
template <typename F, int NH, int T>
__global__ __launch_bounds__(T) void k_init(InitArgs a) {
    constexpr int B = NH * NH * NH;
    constexpr int64_t NV = 8 * B;
    constexpr int S = Lane<NH, T>::S;
    __shared__ MaxwellSmem<F, NH> sm;
    const int64_t c = blockIdx.x;
    double p[5];
    for (int k = 0; k < 5; ++k) p[k] = a.prim ? a.prim[k * a.n + c] : a.prim0[k];
    const double rho = p[0], u[3] = {p[1], p[2], p[3]}, Tt = p[4];
    const Rsrc out = rsrc(static_cast<F *>(a.f_out) + c * NV, uint32_t(NV * sizeof(F)));
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
    relax_store<F, NH, T, false>(sm, zero, F(0), out);
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
        F v[8][1];
        for (int o = 0; o < 8; ++o) v[o][0] = row[o * B + s];
        double s0, sx, sy, sz;
        octant_sums<F, 1>(v, 0, s0, sx, sy, sz);
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

// ---------------------------------------------------------------------------
// configuration table: (NH, threads, waves per EU); every step kernel comes
// with and without non-temporal stores
// ---------------------------------------------------------------------------
#define DVM_STEP_CONFIGS(X) \
    X(2, 64, 4, 0)          \
    X(4, 64, 5, 0)          \
    X(6, 256, 6, 0)         \
    X(6, 64, 4, 0)          \
    X(6, 128, 6, 0)         \
    X(8, 256, 5, 0)         \
    X(8, 64, 3, 0)          \
    X(8, 128, 5, 0)         \
    X(8, 256, 5, 1)         \
    X(8, 512, 4, 0)         \
    X(12, 192, 3, 1)        \
    X(12, 576, 3, 0)        \
    X(12, 576, 5, 1)        \
    X(12, 576, 7, 1)

// reduced kernels (cells without FINER or WALL faces): one shape per N
#define DVM_REG_CONFIGS(X) \
    X(2, 64, 4, 0)         \
    X(4, 64, 5, 0)         \
    X(6, 256, 6, 0)        \
    X(8, 256, 5, 0)        \
    X(12, 192, 3, 1)

// MUSCL step kernels: one shape per N, (NH, threads, waves per EU for FP32
// and for FP64 storage, octant fence)
#define DVM_MUSCL_CONFIGS(X) \
    X(2, 64, 3, 3, 0)        \
    X(4, 64, 3, 3, 0)        \
    X(6, 256, 6, 6, 0)       \
    X(8, 256, 5, 5, 0)       \
    X(12, 576, 7, 3, 1)

template <typename F>
hipError_t step_dispatch(const StepArgs &a, const StepConfig &cfg, hipStream_t st) {
    const dim3 grid(unsigned(a.sel ? a.n_sel : a.n_cells));
    if (cfg.regular) {
        if (!a.sel || a.muscl) return hipErrorInvalidValue;
#define X(NH, T, W, FN)                                                                                     \
        if (a.g.nh == NH && cfg.threads == T && (cfg.wpe == 0 || cfg.wpe == 10 * W + FN)) {                 \
            if (cfg.nt_store) hipLaunchKernelGGL((k_step<F, NH, T, W, FN, true, false, true>), grid, dim3(T), 0, st, a); \
            else hipLaunchKernelGGL((k_step<F, NH, T, W, FN, false, false, true>), grid, dim3(T), 0, st, a); \
            return hipGetLastError();                                                                       \
        }
        DVM_REG_CONFIGS(X)
#undef X
        return hipErrorInvalidValue;
    }
    if (a.muscl) {
        // the shape asked for when the table has it, else the first listed for N
        bool listed = false;
#define X(NH, T, W32, W64, FN) listed |= a.g.nh == NH && cfg.threads == T;
        DVM_MUSCL_CONFIGS(X)
#undef X
#define X(NH, T, W32, W64, FN)                                                                         \
        if (a.g.nh == NH && (!listed || cfg.threads == T)) {                                           \
            constexpr int W = sizeof(F) == 4 ? W32 : W64;                                              \
            hipLaunchKernelGGL((k_step<F, NH, T, W, FN, true, true>), grid, dim3(T), 0, st, a);        \
            return hipGetLastError();                                                                  \
        }
        DVM_MUSCL_CONFIGS(X)
#undef X
        return hipErrorInvalidValue;
    }
#define X(NH, T, W, FN)                                                                       \
    if (a.g.nh == NH && cfg.threads == T && (cfg.wpe == 0 || cfg.wpe == 10 * W + FN)) {        \
        if (cfg.nt_store) hipLaunchKernelGGL((k_step<F, NH, T, W, FN, true>), grid, dim3(T), 0, st, a);  \
        else hipLaunchKernelGGL((k_step<F, NH, T, W, FN, false>), grid, dim3(T), 0, st, a);    \
        return hipGetLastError();                                                             \
    }
    DVM_STEP_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

template <typename F>
hipError_t step_batch_dispatch(const StepArgs *inst, const uint32_t *wg_end, int n_inst, uint32_t total_wg, int nh,
                               const StepConfig &cfg, hipStream_t st) {
    int lg = 0;
    while ((1 << (lg + 1)) <= cfg.xcd_group) ++lg;
    const dim3 grid(total_wg);
#define X(NH, T, W, FN)                                                                                     \
    if (nh == NH && cfg.threads == T && (cfg.wpe == 0 || cfg.wpe == 10 * W + FN)) {                         \
        if (cfg.nt_store)                                                                                   \
            hipLaunchKernelGGL((k_step_batch<F, NH, T, W, FN, true>), grid, dim3(T), 0, st, inst, wg_end, n_inst, lg); \
        else                                                                                                \
            hipLaunchKernelGGL((k_step_batch<F, NH, T, W, FN, false>), grid, dim3(T), 0, st, inst, wg_end, n_inst, lg); \
        return hipGetLastError();                                                                           \
    }
    DVM_STEP_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

inline int step_config_list(int nh, int *threads, int *wpe, int cap) {
    int n = 0;
#define X(NH, T, W, FN)                 \
    if (nh == NH) {                     \
        if (n < cap) {                  \
            threads[n] = T;             \
            wpe[n] = 10 * W + FN;       \
        }                               \
        ++n;                            \
    }
    DVM_STEP_CONFIGS(X)
#undef X
    return n;
}

inline bool reg_config_exists(int nh, int threads, int wpe) {
#define X(NH, T, W, FN) \
    if (nh == NH && threads == T && (wpe == 0 || wpe == 10 * W + FN)) return true;
    DVM_REG_CONFIGS(X)
#undef X
    return false;
}

inline bool step_config_exists(int nh, int threads, int wpe) {
#define X(NH, T, W, FN) \
    if (nh == NH && threads == T && (wpe == 0 || wpe == 10 * W + FN)) return true;
    DVM_STEP_CONFIGS(X)
#undef X
    return false;
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

}  // namespace impl
}  // namespace dvm
