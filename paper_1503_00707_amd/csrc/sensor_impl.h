// sensor_impl.h -- continuum-breakdown sensor, its training, and the
// kinetic/fluid hybrid step (device templates).
//
// Sensor.  Per cell ten features of the local state and its gradients
//   x = [ln rho, u/sqrt(T) (3), ln T, lambda |grad rho|/rho,
//        lambda |grad u_b|/sqrt(T) (3), lambda |grad T|/T],  lambda = tau sqrt(T),
// gradients by central differences over face-neighbour values (the mean of
// the four leaves across a FINER face) with centre distances h, 3h/4 (FINER),
// 3h/2 (COARSER); a domain face uses the cell's own value at distance h.
// The network 10-64-64-1 (exact GELU) maps standardised features to a logit;
// a cell is kinetic iff the logit is > 0 (probability > 1/2).  Inference runs
// on the matrix cores: each wave pushes 16 cells through
// v_mfma_f32_16x16x16_bf16 (BF16 weights and activations, FP32 accumulation).
//
// Training.  FP32 master weights; one thread per sample for the forward and
// backward pass (activations and their GELU derivatives kept in a scratch
// block), weight gradients summed in FP64 in sample order (deterministic),
// then Adam.  Loss: class-weighted binary cross-entropy on the logit.
//
// Hybrid step (paper: kinetic and continuum cells on one adaptive mesh).  A
// frozen mask per step: kinetic cells run the fused DVM step unchanged;
// fluid cells carry only U = (rho, rho u, E) (the moments buffer) and advance
//   U' = U - dt/h sum_faces (H_out(Mt(U)) + H_in(g_nb)),
// H the half-range flux sums w sum_{+-xi.n > 0} (xi.n) psi g of the discrete
// velocity set, g_nb = f (kinetic neighbour, summed over its half row) or
// Mt(U_nb) (fluid neighbour, from separable 1D sums of its Maxwellian
// tables: O(N) per face instead of O(N^3)).  Fluid cells next to kinetic
// cells (and cells turning kinetic) write Mt(U) into the state buffer first,
// so the kinetic transport reads them as ordinary rows.
#pragma once

#include "step_impl.h"

namespace dvm {
namespace impl {

// parameter block of the network (floats)
constexpr int kIn = 10, kHid = 64;
constexpr int kW1 = 0, kB1 = kW1 + kHid * kIn, kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid, kW3 = kB2 + kHid;
constexpr int kB3 = kW3 + kHid, kMean = kB3 + 1, kStd = kMean + kIn, kParams = kStd + kIn;
constexpr int kWeights = kMean;
static_assert(kParams == 4949 && kWeights == 4929, "parameter block layout");

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------

struct FeatArgs {
    const double *mom;   // [5][n]
    const DevCell *cells;
    int64_t n;
    double h0;
    int tau_mode;
    double tau_or_kn;
};

__device__ inline void prim5(const double *mom, int64_t n, int64_t c, double q[5]) {
    const double rho = mom[c];
    const double ux = mom[n + c] / rho, uy = mom[2 * n + c] / rho, uz = mom[3 * n + c] / rho;
    q[0] = rho;
    q[1] = ux;
    q[2] = uy;
    q[3] = uz;
    q[4] = (2.0 * mom[4 * n + c] / rho - ((ux * ux + uy * uy) + uz * uz)) / 3.0;
}

// features of cell c (FP64)
__device__ inline void cell_features(const FeatArgs &a, int64_t c, double x[10]) {
    const DevCell &cell = a.cells[c];
    const double h = a.h0 / double(1 << cell.level);
    double q[5];
    prim5(a.mom, a.n, c, q);
    double g2[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double qs[2][5], ds[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int f = 2 * b + side;
            const int ty = cell.type[f];
            ds[side] = h;
            if (ty == DVM_FACE_SAME || ty == DVM_FACE_COARSER) {
                prim5(a.mom, a.n, cell.nbr[f][0], qs[side]);
                if (ty == DVM_FACE_COARSER) ds[side] = 1.5 * h;
            } else if (ty == DVM_FACE_FINER) {
                double t[4][5];
                for (int k = 0; k < 4; ++k) prim5(a.mom, a.n, cell.nbr[f][k], t[k]);
                for (int v = 0; v < 5; ++v) qs[side][v] = 0.25 * (((t[0][v] + t[1][v]) + t[2][v]) + t[3][v]);
                ds[side] = 0.75 * h;
            } else {
                for (int v = 0; v < 5; ++v) qs[side][v] = q[v];
            }
        }
        for (int v = 0; v < 5; ++v) {
            const double d = (qs[1][v] - qs[0][v]) / (ds[0] + ds[1]);
            g2[v] += d * d;
        }
    }
    const double rho = q[0], T = q[4], sT = sqrt(T);
    const double tau = a.tau_mode == DVM_TAU_HS ? a.tau_or_kn / (rho * sT) : a.tau_or_kn;
    const double lam = tau * sT;
    x[0] = log(rho);
    x[1] = q[1] / sT;
    x[2] = q[2] / sT;
    x[3] = q[3] / sT;
    x[4] = log(T);
    x[5] = lam * sqrt(g2[0]) / rho;
    x[6] = lam * sqrt(g2[1]) / sT;
    x[7] = lam * sqrt(g2[2]) / sT;
    x[8] = lam * sqrt(g2[3]) / sT;
    x[9] = lam * sqrt(g2[4]) / T;
}

__global__ __launch_bounds__(256) void k_features(FeatArgs a, float *x) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= a.n) return;
    double f[10];
    cell_features(a, c, f);
    for (int k = 0; k < 10; ++k) x[c * 10 + k] = float(f[k]);
}

// ---------------------------------------------------------------------------
// labels: r = |f - Mt|_2 / |Mt|_2 per cell, Mt of the cell's own moments
// ---------------------------------------------------------------------------

template <typename F, int NH, int T>
__global__ __launch_bounds__(T) void k_labels(const F *f, float *r, VelGrid g) {
    using L = Lane<NH, T>;
    constexpr int S = L::S;
    constexpr int64_t NV = 8 * L::B;
    __shared__ StepSmem<F, NH, T> sm;
    const L ln;
    const int64_t c = blockIdx.x;
    const F *row = f + c * NV;
    F fo[8][S];
    double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < S; ++q) {
#pragma unroll
        for (int o = 0; o < 8; ++o) fo[o][q] = ln.ok(q) ? row[o * L::B + ln.slot(q)] : F(0);
        if (!ln.ok(q)) continue;
        int a3[3];
        ln.axes(q, a3[0], a3[1], a3[2]);
        const double xa = (a3[0] + 0.5) * g.dv[0], ya = (a3[1] + 0.5) * g.dv[1], za = (a3[2] + 0.5) * g.dv[2];
        double s0, sx, sy, sz;
        octant_sums<F, S>(fo, q, s0, sx, sy, sz);
        m[0] += s0;
        m[1] += xa * sx;
        m[2] += ya * sy;
        m[3] += za * sz;
        m[4] += 0.5 * (xa * xa + ya * ya + za * za) * s0;
    }
    block_sum<T, 5>(m, sm.red);
    const double w = g.w;
    const double rho = w * m[0];
    const double u[3] = {w * m[1] / rho, w * m[2] / rho, w * m[3] / rho};
    const double Tt = (2.0 * w * m[4] / rho - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / 3.0;
    maxwell_tables<F, NH, T>(sm.mx, rho, u, Tt, 1.0, g);
    double s2[2] = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < S; ++q) {
        if (!ln.ok(q)) continue;
        int a3[3];
        ln.axes(q, a3[0], a3[1], a3[2]);
        double G[3][2], P[3][2];
        for (int b = 0; b < 3; ++b) {
            G[b][0] = sm.mx.tab[b][NH - 1 - a3[b]][0];
            G[b][1] = sm.mx.tab[b][NH + a3[b]][0];
            P[b][0] = sm.mx.tab[b][NH - 1 - a3[b]][1];
            P[b][1] = sm.mx.tab[b][NH + a3[b]][1];
        }
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int ox = o >> 2, oy = (o >> 1) & 1, oz = o & 1;
            const double M = (G[0][ox] * G[1][oy]) * G[2][oz] * ((P[0][ox] + P[1][oy]) + P[2][oz]);
            const double d = double(fo[o][q]) - M;
            s2[0] += d * d;
            s2[1] += M * M;
        }
    }
    block_sum<T, 2>(s2, sm.red);
    if (threadIdx.x == 0) r[c] = float(sqrt(s2[0] / s2[1]));
}

// ---------------------------------------------------------------------------
// the network: FP32 reference forward, BF16 matrix-core forward
// ---------------------------------------------------------------------------

// one sample, FP32, weights in LDS
__device__ inline float mlp_logit32(const float *w, const float *xr) {
    float xs[kIn];
    for (int k = 0; k < kIn; ++k) xs[k] = (xr[k] - w[kMean + k]) / w[kStd + k];
    float h1[kHid];
    for (int j = 0; j < kHid; ++j) {
        float z = w[kB1 + j];
        for (int k = 0; k < kIn; ++k) z += w[kW1 + j * kIn + k] * xs[k];
        h1[j] = gelu_f(z);
    }
    float out = w[kB3];
    for (int j = 0; j < kHid; ++j) {
        float z = w[kB2 + j];
        for (int k = 0; k < kHid; ++k) z += w[kW2 + j * kHid + k] * h1[k];
        out += w[kW3 + j] * gelu_f(z);
    }
    return out;
}

__global__ __launch_bounds__(256) void k_mlp_fwd32(const float *P, const float *x, int64_t n, float *z) {
    __shared__ float w[kParams];
    for (int i = threadIdx.x; i < kParams; i += 256) w[i] = P[i];
    __syncthreads();
    const int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (s >= n) return;
    z[s] = mlp_logit32(w, x + s * kIn);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float v) {
    uint32_t u = __builtin_bit_cast(uint32_t, v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return short(u >> 16);
}

// Logits of R rows per workgroup (R / 16 waves x 16 rows) on the matrix cores.
// Operand layout of v_mfma_f32_16x16x16_bf16 for lane l: A[i = l % 16][k =
// 4 (l / 16) + 0..3], B[k = 4 (l / 16) + 0..3][j = l % 16], result
// D[i = 4 (l / 16) + v][j = l % 16], v = 0..3.  Hidden activations go through
// LDS to turn the result layout into the next layer's A layout.
// xs: standardised features [R][16] (columns >= 10 are zero), written by the
// caller into LDS; out: logits of the R rows.
template <int R>
__device__ inline void mlp_tile_mfma(const float *w, const float (&xs)[R][16], float (&h1)[R / 16][16][kHid + 4],
                                     float *out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    // layer 1: K = 16 (features padded), 4 column blocks of 16
    bf16x4 a;
    for (int t = 0; t < 4; ++t) a[t] = to_bf16(xs[wv * 16 + li][4 * lg + t]);
    for (int nb = 0; nb < 4; ++nb) {
        const int j = nb * 16 + li;
        bf16x4 b;
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * lg + t;
            b[t] = to_bf16(k < kIn ? w[kW1 + j * kIn + k] : 0.0f);
        }
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, d, 0, 0, 0);
        for (int v = 0; v < 4; ++v) h1[wv][4 * lg + v][j] = gelu_f(d[v] + w[kB1 + j]);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    // layer 2: K = 64 in 4 steps, 4 column blocks; layer 3 as a lane reduction
    float part[4] = {0.f, 0.f, 0.f, 0.f};
    for (int nb = 0; nb < 4; ++nb) {
        const int j = nb * 16 + li;
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        for (int kb = 0; kb < 4; ++kb) {
            bf16x4 a2, b2;
            for (int t = 0; t < 4; ++t) {
                const int k = kb * 16 + 4 * lg + t;
                a2[t] = to_bf16(h1[wv][li][k]);
                b2[t] = to_bf16(w[kW2 + j * kHid + k]);
            }
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, b2, d, 0, 0, 0);
        }
        const float w3 = w[kW3 + j];
        for (int v = 0; v < 4; ++v) part[v] += w3 * gelu_f(d[v] + w[kB2 + j]);
    }
    // sum over the 16 lanes of a group (same rows, different columns)
    for (int v = 0; v < 4; ++v)
        for (int off = 1; off < 16; off <<= 1) part[v] += __shfl_xor(part[v], off, 64);
    if (li == 0)
        for (int v = 0; v < 4; ++v) out[wv * 16 + 4 * lg + v] = part[v] + w[kB3];
}

// Logits of raw feature rows x[n][10] on the matrix cores.
__global__ __launch_bounds__(256) void k_mlp_fwd_mfma(const float *P, const float *x, int64_t n, float *z) {
    __shared__ float w[kParams];
    __shared__ float xs[64][16];
    __shared__ float h1[4][16][kHid + 4];
    __shared__ float out[64];
    for (int i = threadIdx.x; i < kParams; i += 256) w[i] = P[i];
    __syncthreads();
    const int64_t r0 = int64_t(blockIdx.x) * 64;
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
        const int r = e >> 4, k = e & 15;
        const int64_t s = r0 + r;
        xs[r][k] = (k < kIn && s < n) ? (x[s * kIn + k] - w[kMean + k]) / w[kStd + k] : 0.0f;
    }
    __syncthreads();
    mlp_tile_mfma<64>(w, xs, h1, out);
    __syncthreads();
    if (threadIdx.x < 64 && r0 + threadIdx.x < n) z[r0 + threadIdx.x] = out[threadIdx.x];
}

// Copy the parameter block to LDS with NT threads: 16-byte loads, all in
// flight before the first LDS store (a 64-thread workgroup would otherwise
// wait out some 80 dependent round trips); element loads when P is not
// 16-byte aligned.  w must be 16-byte aligned.  The tail lanes re-read the
// last vector instead of branching around the load, which keeps the staging
// registers out of scratch.
template <int NT>
__device__ inline void stage_params(float *w, const float *P) {
    constexpr int n4 = kParams / 4, per = (n4 + NT - 1) / NT;
    if ((reinterpret_cast<uintptr_t>(P) & 15) == 0) {
        const float4 *P4 = reinterpret_cast<const float4 *>(P);
        float4 *w4 = reinterpret_cast<float4 *>(w);
        float4 r[per];
#pragma unroll
        for (int k = 0; k < per; ++k) r[k] = P4[min(int(threadIdx.x) + k * NT, n4 - 1)];
#pragma unroll
        for (int k = 0; k < per; ++k) {
            const int i = threadIdx.x + k * NT;
            if (i < n4) w4[i] = r[k];
        }
        for (int i = 4 * n4 + threadIdx.x; i < kParams; i += NT) w[i] = P[i];
    } else {
        for (int i = threadIdx.x; i < kParams; i += NT) w[i] = P[i];
    }
}

// The sensor: features of R cells per workgroup (one thread each; the
// workgroup has R / 16 waves), then the network on the matrix cores
// (mlp != nullptr) or the largest gradient-length Knudsen number against
// kappa.  mask = 1: kinetic.  R = 16 spreads a small mesh over more compute
// units; a row's result does not depend on R.
template <int R>
__global__ __launch_bounds__(4 * R) void k_sensor(FeatArgs a, const float *P, double kappa, uint8_t *mask,
                                                  float *score) {
    static_assert(R == 16 || R == 64, "rows per workgroup");
    __shared__ __align__(16) float w[kParams];
    __shared__ float xs[R][16];
    __shared__ float h1[R / 16][16][kHid + 4];
    __shared__ float out[R];
    const int64_t c0 = int64_t(blockIdx.x) * R;
    if (P) stage_params<4 * R>(w, P);
    __syncthreads();
    if (threadIdx.x < R) {
        const int64_t c = c0 + threadIdx.x;
        double f[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (c < a.n) cell_features(a, c, f);
        if (P) {
            for (int k = 0; k < 16; ++k)
                xs[threadIdx.x][k] = (k < kIn && c < a.n) ? (float(f[k]) - w[kMean + k]) / w[kStd + k] : 0.0f;
        } else {
            double g = f[5];
            for (int k = 6; k < 10; ++k) g = f[k] > g ? f[k] : g;
            out[threadIdx.x] = float(g);
        }
    }
    __syncthreads();
    if (P) mlp_tile_mfma<R>(w, xs, h1, out);
    __syncthreads();
    if (threadIdx.x < R) {
        const int64_t c = c0 + threadIdx.x;
        if (c < a.n) {
            const float v = out[threadIdx.x];
            if (score) score[c] = P ? 1.0f / (1.0f + expf(-v)) : v;
            mask[c] = P ? uint8_t(v > 0.0f) : uint8_t(double(v) > kappa);
        }
    }
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------

// per-sample scratch record (floats)
constexpr int kRx = 0, kRh1 = kRx + kIn, kRg1 = kRh1 + kHid, kRh2 = kRg1 + kHid, kRd1 = kRh2 + kHid;
constexpr int kRd2 = kRd1 + kHid, kRdz = kRd2 + kHid, kRec = kRdz + 1;

// forward and backward of one sample per thread; block partial losses
__global__ __launch_bounds__(256) void k_train_fb(const float *P, const float *x, const float *y, int64_t n,
                                                  float pos_weight, float *rec, double *loss_part) {
    __shared__ float w[kParams];
    __shared__ double red[4];
    for (int i = threadIdx.x; i < kParams; i += 256) w[i] = P[i];
    __syncthreads();
    const int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double loss = 0.0;
    if (s < n) {
        float *R = rec + s * kRec;
        for (int k = 0; k < kIn; ++k) R[kRx + k] = (x[s * kIn + k] - w[kMean + k]) / w[kStd + k];
        for (int j = 0; j < kHid; ++j) {
            float z = w[kB1 + j];
            for (int k = 0; k < kIn; ++k) z += w[kW1 + j * kIn + k] * R[kRx + k];
            R[kRh1 + j] = gelu_f(z);
            R[kRg1 + j] = gelu_d(z);
        }
        float zo = w[kB3];
        for (int j = 0; j < kHid; ++j) {
            float z = w[kB2 + j];
            for (int k = 0; k < kHid; ++k) z += w[kW2 + j * kHid + k] * R[kRh1 + k];
            R[kRh2 + j] = gelu_f(z);
            R[kRd2 + j] = gelu_d(z);  // derivative for now, delta below
            zo += w[kW3 + j] * R[kRh2 + j];
        }
        const float yy = y[s];
        const float wt = yy > 0.5f ? pos_weight : 1.0f;
        const float ez = expf(-fabsf(zo));
        const float sig = zo >= 0.0f ? 1.0f / (1.0f + ez) : ez / (1.0f + ez);
        loss = double(wt) * (double(fmaxf(zo, 0.0f)) - double(zo) * yy + log1p(double(ez)));
        const float dz = wt * (sig - yy) / float(n);
        R[kRdz] = dz;
        for (int j = 0; j < kHid; ++j) R[kRd2 + j] = dz * w[kW3 + j] * R[kRd2 + j];
        for (int k = 0; k < kHid; ++k) {
            float acc = 0.0f;
            for (int j = 0; j < kHid; ++j) acc += R[kRd2 + j] * w[kW2 + j * kHid + k];
            R[kRd1 + k] = acc * R[kRg1 + k];
        }
    }
    double v[1] = {loss};
    block_sum<256, 1>(v, red);
    if (threadIdx.x == 0) loss_part[blockIdx.x] = v[0];
}

// weight gradients (FP64 sums in sample order) and the mean loss
__global__ __launch_bounds__(256) void k_train_grads(const float *rec, int64_t n, const double *loss_part, int nlp,
                                                     float *grad, double *loss) {
    const int i = int(blockIdx.x) * 256 + threadIdx.x;
    if (i == 0) {
        double l = 0.0;
        for (int b = 0; b < nlp; ++b) l += loss_part[b];
        *loss = l / double(n);
    }
    if (i >= kWeights) return;
    int a, b;  // gradient = sum_s R[a] * R[b] (b < 0: sum_s R[a])
    if (i < kB1) {
        a = kRd1 + (i - kW1) / kIn;
        b = kRx + (i - kW1) % kIn;
    } else if (i < kW2) {
        a = kRd1 + (i - kB1);
        b = -1;
    } else if (i < kB2) {
        a = kRd2 + (i - kW2) / kHid;
        b = kRh1 + (i - kW2) % kHid;
    } else if (i < kW3) {
        a = kRd2 + (i - kB2);
        b = -1;
    } else if (i < kB3) {
        a = kRdz;
        b = kRh2 + (i - kW3);
    } else {
        a = kRdz;
        b = -1;
    }
    double g = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        const float *R = rec + s * kRec;
        g += b < 0 ? double(R[a]) : double(R[a]) * double(R[b]);
    }
    grad[i] = float(g);
}

// Adam with bias correction; c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ __launch_bounds__(256) void k_adam(float *P, float *m, float *v, const float *grad, float lr, float c1,
                                              float c2) {
    const int i = int(blockIdx.x) * 256 + threadIdx.x;
    if (i >= kWeights) return;
    const float g = grad[i];
    const float mi = 0.9f * m[i] + 0.1f * g;
    const float vi = 0.999f * v[i] + 0.001f * g * g;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// standardisation statistics of a feature set (FP64, fixed order)
__global__ __launch_bounds__(256) void k_norm_stats(const float *x, int64_t n, float *P) {
    __shared__ double red[4 * 2];
    const int k = blockIdx.x;  // feature
    double s[2] = {0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += 256) s[0] += double(x[i * kIn + k]);
    double v1[1] = {s[0]};
    block_sum<256, 1>(v1, red);
    const double mean = v1[0] / double(n);
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double d = double(x[i * kIn + k]) - mean;
        s[1] += d * d;
    }
    double v2[1] = {s[1]};
    block_sum<256, 1>(v2, red);
    if (threadIdx.x == 0) {
        const double sd = sqrt(v2[0] / double(n));
        P[kMean + k] = float(mean);
        P[kStd + k] = float(sd > 1e-6 ? sd : 1e-6);
    }
}

// ---------------------------------------------------------------------------
// hybrid step
// ---------------------------------------------------------------------------

// per axis: full A[3], B[3]; + half A[4], B[4]; - half A[4], B[4]; then rho, u[3], T
constexpr int kFluxRec = 71;

struct HybArgs {
    const uint8_t *mask;  // effective mask (1 kinetic)
    uint8_t *prev;        // mask of the previous hybrid step
    uint8_t *rows;        // bit 0: write Mt(U) into the state buffer before the step;
                          // bit 1: a kinetic cell with a fluid face neighbour
    double *flux;         // [n][kFluxRec] separable sums of fluid cells' Maxwellians
    double *face;         // [n][6][5] outgoing half-range fluxes of kinetic cells next to fluid ones
    int32_t closed;       // fluid-fluid faces: continuous half-range integrals (erf form)
    int32_t pad;
};

// mask | (cell touches a non-periodic domain face): those cells stay kinetic
__global__ __launch_bounds__(256) void k_mask_eff(const uint8_t *in, uint8_t *out, const DevCell *cells, int64_t n) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= n) return;
    uint8_t m = in[c] ? 1 : 0;
    for (int f = 0; f < 6; ++f) m |= uint8_t(cells[c].type[f] >= DVM_FACE_INFLOW);
    out[c] = m;
}

// Corrected Maxwellian of conserved moments U by one thread (the same
// construction as maxwell_solve): C and the coefficients d of the centred
// basis.  Returns false for a non-physical state.
__device__ inline bool maxwell_serial(const double U[5], const VelGrid &g, double u[3], double &sT, double &C,
                                      double d[5]) {
    const int nh = g.nh, N = 2 * nh;
    const double rho = U[0];
    for (int b = 0; b < 3; ++b) u[b] = U[1 + b] / rho;
    const double Tt = (2.0 * U[4] / rho - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / 3.0;
    if (!(rho > 0.0) || !(Tt > 0.0)) return false;
    sT = sqrt(Tt);
    double S[15];
    for (int b = 0; b < 3; ++b) {
        double p[5] = {0, 0, 0, 0, 0};
        const double dvb = b == 0 ? g.dv[0] : b == 1 ? g.dv[1] : g.dv[2];
        const double ub = b == 0 ? u[0] : b == 1 ? u[1] : u[2];
        for (int k = 0; k < N; ++k) {
            const double ck = ((double(k - nh) + 0.5) * dvb - ub) / sT;
            double t = exp(-0.5 * ck * ck);
            for (int q = 0; q < 5; ++q) {
                p[q] += t;
                t *= ck;
            }
        }
        for (int q = 0; q < 5; ++q) S[5 * b + q] = p[q] * dvb;
    }
    const double x2 = 6.283185307179586476925286766559 * Tt;
    C = rho / (x2 * sqrt(x2));
    double A[5][6];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 6; ++j) {
            if (j < 5) A[i][j] = gram_entry(i, j, &S[0], &S[5], &S[10]);
            else A[i][j] = (i == 0 ? 1.0 : i == 4 ? 3.0 : 0.0) * (rho / C) - gram_entry(i, 0, &S[0], &S[5], &S[10]);
        }
    for (int k = 0; k < 5; ++k)
        for (int i = 0; i < 5; ++i) {
            if (i == k) continue;
            const double r = A[i][k] / A[k][k];
            for (int j = 0; j < 6; ++j) A[i][j] -= r * A[k][j];
        }
    for (int i = 0; i < 5; ++i) d[i] = A[i][5] / A[i][i];
    return true;
}

// Per cell, one thread: fluid cells get the separable sums of their
// Maxwellian; the cells whose state buffer row must hold Mt(U) this step
// are flagged (fluid cells next to a kinetic one, cells turning kinetic),
// and so are the kinetic cells next to a fluid one (the step kernel reads
// that one byte instead of its neighbours' masks); the previous mask is
// updated.
__global__ __launch_bounds__(256) void k_fluid_state(StepArgs a, HybArgs h) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x, n = a.n_cells;
    if (c >= n) return;
    const int m = h.mask[c], pm = h.prev[c];
    const DevCell &cell = a.cells[c];
    bool kin_nb = false, fluid_nb = false;
    for (int f = 0; f < 6; ++f) {
        const int ty = cell.type[f];
        const int k = ty == DVM_FACE_FINER ? 4 : (ty == DVM_FACE_SAME || ty == DVM_FACE_COARSER) ? 1 : 0;
        for (int q = 0; q < k; ++q) {
            const bool kin = h.mask[cell.nbr[f][q]] != 0;
            kin_nb |= kin;
            fluid_nb |= !kin;
        }
    }
    h.rows[c] = uint8_t(((m == 0 && kin_nb) || (m == 1 && pm == 0)) | ((m == 1 && fluid_nb) ? 2 : 0));
    h.prev[c] = uint8_t(m);
    if (m) return;
    double U[5], u[3], sT, C, d[5];
    for (int x = 0; x < 5; ++x) U[x] = a.mom[x * n + c];
    if (!maxwell_serial(U, a.g, u, sT, C, d)) {
        *a.flag = 1;
        return;
    }
    const int nh = a.g.nh, N = 2 * nh;
    double *R = h.flux + c * kFluxRec;
    {
        // the primitive state of U itself (the closed-form fluxes)
        const double rho = U[0], v0 = U[1] / rho, v1 = U[2] / rho, v2 = U[3] / rho;
        R[66] = rho;
        R[67] = v0;
        R[68] = v1;
        R[69] = v2;
        R[70] = (2.0 * U[4] / rho - ((v0 * v0 + v1 * v1) + v2 * v2)) / 3.0;
    }
    for (int b = 0; b < 3; ++b) {
        double acc[22];
        for (int t = 0; t < 22; ++t) acc[t] = 0.0;
        const double dvb = b == 0 ? a.g.dv[0] : b == 1 ? a.g.dv[1] : a.g.dv[2];
        const double ub = b == 0 ? u[0] : b == 1 ? u[1] : u[2];
        const double db = b == 0 ? d[1] : b == 1 ? d[2] : d[3];
        for (int k = 0; k < N; ++k) {
            const double xi = (double(k - nh) + 0.5) * dvb;
            const double cc = (xi - ub) / sT;
            const double gk = exp(-0.5 * cc * cc);
            const double G = b == 0 ? gk * C : gk;
            const double P = (b == 0 ? 1.0 + d[0] : 0.0) + db * cc + d[4] * cc * cc;
            const int hb = k >= nh ? 6 : 14;
            double xp = 1.0;
            for (int p = 0; p < 4; ++p) {
                if (p < 3) {
                    acc[p] += xp * G;
                    acc[3 + p] += xp * G * P;
                }
                acc[hb + p] += xp * G;
                acc[hb + 4 + p] += xp * G * P;
                xp *= xi;
            }
        }
        for (int t = 0; t < 22; ++t) R[b * 22 + t] = acc[t];
    }
}

// Mt(U) rows of the flagged cells (one workgroup per cell, others exit).
template <typename F, int NH, int T>
__global__ __launch_bounds__(T) void k_hybrid_rows(StepArgs a, HybArgs h) {
    constexpr int64_t NV = 8 * NH * NH * NH;
    __shared__ MaxwellSmem<F, NH> sm;
    const int64_t c = blockIdx.x, n = a.n_cells;
    if (!(h.rows[c] & 1)) return;
    const double rho = a.mom[c];
    const double u[3] = {a.mom[n + c] / rho, a.mom[2 * n + c] / rho, a.mom[3 * n + c] / rho};
    const double Tt = (2.0 * a.mom[4 * n + c] / rho - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / 3.0;
    if (!(rho > 0.0) || !(Tt > 0.0)) {
        if (threadIdx.x == 0) *a.flag = 1;
        return;
    }
    maxwell_tables<F, NH, T>(sm, rho, u, Tt, 1.0, a.g);
    F zero[8][Lane<NH, T>::S];
    for (int q = 0; q < Lane<NH, T>::S; ++q)
        for (int o = 0; o < 8; ++o) zero[o][q] = F(0);
    const Rsrc out = rsrc(static_cast<const F *>(a.f_in) + c * NV, uint32_t(NV * sizeof(F)));
    relax_store<F, NH, T, false>(sm, zero, F(0), out);
}

// sum over the tensor grid of prod_a xi_a^p[a] Mt, the normal axis b summed
// over one half (hs = 6: positive, 14: negative), the others over all nodes
__device__ __forceinline__ double sep_moment(const double *R, int b, int hs, int px, int py, int pz) {
    const double *X = R, *Y = R + 22, *Z = R + 44;
    const double Ax = b == 0 ? X[hs + px] : X[px], Bx = b == 0 ? X[hs + 4 + px] : X[3 + px];
    const double Ay = b == 1 ? Y[hs + py] : Y[py], By = b == 1 ? Y[hs + 4 + py] : Y[3 + py];
    const double Az = b == 2 ? Z[hs + pz] : Z[pz], Bz = b == 2 ? Z[hs + 4 + pz] : Z[3 + pz];
    return Bx * Ay * Az + Ax * By * Az + Ax * Ay * Bz;
}

// w sum over one half (normal axis b) of xi_b psi Mt, psi = (1, xi, |xi|^2/2)
__device__ __forceinline__ void sep_flux(const double *R, int b, int hs, double w, double out[5]) {
    const int px = b == 0, py = b == 1, pz = b == 2;
    out[0] = w * sep_moment(R, b, hs, px, py, pz);
    out[1] = w * sep_moment(R, b, hs, px + 1, py, pz);
    out[2] = w * sep_moment(R, b, hs, px, py + 1, pz);
    out[3] = w * sep_moment(R, b, hs, px, py, pz + 1);
    out[4] = 0.5 * w *
             ((sep_moment(R, b, hs, px + 2, py, pz) + sep_moment(R, b, hs, px, py + 2, pz)) +
              sep_moment(R, b, hs, px, py, pz + 2));
}

// Kinetic cells next to fluid ones: the half-range flux of their own f
// through each such face, w sum_{leaving} xi_b psi f (signed xi_b), before
// the transport overwrites f.
struct HybHook {
    HybArgs h;
    // moments of the values leaving through face FACE (its axis and side
    // compile-time constants, so the octants it selects are static)
    template <int FACE, typename F, int NH, int T>
    __device__ __forceinline__ void face_flux(const StepArgs &a, int64_t c, const Regs<F, NH, T> &fo,
                                              double *red) const {
        using L = Lane<NH, T>;
        constexpr int S = L::S;
        constexpr int b = FACE >> 1, side = FACE & 1;
        const L ln;
        // For a round the four leaving octants share |xi| and the sign along
        // b; only the signs along the other two axes (p, r) change.  So the
        // five moments need three sums of the stored values, formed in the
        // storage precision and widened once: S (all four), Sp and Sr (signed
        // by the sign along p and along r).
        constexpr int p = b == 0 ? 1 : 0, r = b == 2 ? 1 : 2;
        const double sg = side ? 1.0 : -1.0;
        double v[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < S; ++q) {
            if (!ln.ok(q)) continue;
            F s0 = F(0), sp = F(0), sr = F(0);
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int sgn[3] = {o >> 2, (o >> 1) & 1, o & 1};
                if (sgn[b] != side) continue;  // not leaving through FACE
                const F x = fo[o][q];
                s0 += x;
                sp += sgn[p] ? x : -x;
                sr += sgn[r] ? x : -x;
            }
            int a3[3];
            ln.axes(q, a3[0], a3[1], a3[2]);
            const double ab[3] = {(a3[0] + 0.5) * a.g.dv[0], (a3[1] + 0.5) * a.g.dv[1], (a3[2] + 0.5) * a.g.dv[2]};
            const double S0 = double(s0), Sp = double(sp), Sr = double(sr);
            const double xb = sg * ab[b];  // xi . e_b of the leaving values
            v[0] += xb * S0;
            v[1 + b] += xb * xb * S0;
            v[1 + p] += xb * ab[p] * Sp;
            v[1 + r] += xb * ab[r] * Sr;
            v[4] += 0.5 * xb * ((ab[0] * ab[0] + ab[1] * ab[1]) + ab[2] * ab[2]) * S0;
        }
        block_sum<T, 5>(v, red);
        if (threadIdx.x == 0)
            for (int x = 0; x < 5; ++x) h.face[(c * 6 + FACE) * 5 + x] = a.g.w * v[x];
    }
    template <typename F, int NH, int T>
    __device__ __forceinline__ void apply(const StepArgs &a, const CellView &cell, int64_t c,
                                          const Regs<F, NH, T> &fo, double *red) const {
#pragma nounroll
        for (int f = 0; f < 6; ++f) {
            const int ty = cell.type_rt(f);
            const int k = ty == DVM_FACE_FINER ? 4 : (ty == DVM_FACE_SAME || ty == DVM_FACE_COARSER) ? 1 : 0;
            bool fluid_nb = false;
            for (int q = 0; q < k; ++q) fluid_nb |= h.mask[cell.nbr_rt(f, q)] == 0;
            if (!fluid_nb) continue;
            switch (f) {
            case 0: face_flux<0, F, NH, T>(a, c, fo, red); break;
            case 1: face_flux<1, F, NH, T>(a, c, fo, red); break;
            case 2: face_flux<2, F, NH, T>(a, c, fo, red); break;
            case 3: face_flux<3, F, NH, T>(a, c, fo, red); break;
            case 4: face_flux<4, F, NH, T>(a, c, fo, red); break;
            default: face_flux<5, F, NH, T>(a, c, fo, red); break;
            }
        }
    }
};

// Kinetic cells (fluid cells: k_fluid_update), in the XCD-aware cell order
// of the plain step.  A kinetic cell with no fluid face neighbour has nothing
// to record and runs exactly the plain step's code (the reduced code when it
// has no FINER or WALL face); one next to a fluid cell runs the full code with
// the interface-flux hook.  All three compute the same step, bitwise.
template <typename F, int NH, int T, int WPE, int FENCE, bool NT>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_step_hybrid(StepArgs a,
                                                                                               HybArgs h) {
    __shared__ StepSmem<F, NH, T> sm;
    const int64_t c = remap_cell(blockIdx.x, gridDim.x, a.xcd_log2);
    if (!h.mask[c]) return;
    // one byte, written by k_fluid_state: whether a face neighbour is fluid
    if (h.rows[c] & 2) {
        const HybHook hook{h};
        step_cell<F, NH, T, FENCE, NT, false, false, HybHook>(a, c, sm, hook);
    } else if (needs_correction(a.cells, c)) {
        step_cell<F, NH, T, FENCE, NT, false, false>(a, c, sm);
    } else {
        step_cell<F, NH, T, FENCE, NT, false, true>(a, c, sm);
    }
}

// Half-range flux of the continuous Maxwellian of (rho, u, T) = P[0..4]
// through a face with normal e_b: the integral over xi_b > 0 (pos) or < 0 of
// xi_b (1, xi, |xi|^2 / 2) M.  With xi_b = u_b + sqrt(T) t, t standard
// normal, the half-space is t > -s (pos) or t < -s, s = u_b / sqrt(T); its
// probability is q = erfc(-+s / sqrt 2) / 2 and the truncated moments of t
// follow from phi(s) = exp(-s^2/2) / sqrt(2 pi): E[t] = +-phi,
// E[t^2] = q -+ s phi, E[t^3] = +-(s^2 + 2) phi.  The transverse axes are
// full Gaussians (mean u_a, variance T).
__device__ __forceinline__ void closed_flux(const double *P, int b, bool pos, double out[5]) {
    const double rho = P[0], T = P[4], sd = sqrt(T);
    const double ub = P[1 + b], s = ub / sd;
    const double sg = pos ? 1.0 : -1.0;
    const double q = 0.5 * erfc(-sg * s * 0.70710678118654752440);
    const double ph = exp(-0.5 * s * s) * 0.39894228040143267794;
    const double m1 = ub * q + sg * sd * ph;
    const double m2 = (ub * ub + T) * q + sg * ub * sd * ph;
    const double m3 = (ub * ub + 3.0 * T) * ub * q + sg * (ub * ub + 2.0 * T) * sd * ph;
    double tr = 0.0;
    for (int x = 0; x < 3; ++x) {
        if (x == b) {
            out[1 + x] = rho * m2;
        } else {
            out[1 + x] = rho * P[1 + x] * m1;
            tr += P[1 + x] * P[1 + x] + T;
        }
    }
    out[0] = rho * m1;
    out[4] = 0.5 * rho * (m3 + m1 * tr);
}

// Fluid cells, one thread each: U' = U - dt/h sum_faces (H_out + H_in).
__global__ __launch_bounds__(256) void k_fluid_update(StepArgs a, HybArgs h) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x, n = a.n_cells;
    if (c >= n || h.mask[c]) return;
    const DevCell &cell = a.cells[c];
    const double hc = a.h0 / double(1 << cell.level);
    const double w = a.g.w;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int f = 0; f < 6; ++f) {
        const int b = f >> 1, side = f & 1;
        const double sg = side ? 1.0 : -1.0;  // outward normal along b
        const int ty = cell.type[f];
        double hout[5];
        sep_flux(h.flux + c * kFluxRec, b, side ? 6 : 14, w, hout);
        const int nk = ty == DVM_FACE_FINER ? 4 : 1;
        if (h.closed) {
            // per neighbour: closed-form fluxes on both sides of a fluid-fluid
            // face, the discrete ones where the neighbour is kinetic
            double cout[5], s[5] = {0, 0, 0, 0, 0};
            closed_flux(h.flux + c * kFluxRec + 66, b, side == 1, cout);
            for (int k = 0; k < nk; ++k) {
                const int64_t nb = cell.nbr[f][k];
                double t[5];
                if (h.mask[nb] == 0) {
                    closed_flux(h.flux + nb * kFluxRec + 66, b, side == 0, t);
                    for (int x = 0; x < 5; ++x) s[x] += cout[x] + t[x];
                } else {
                    const double *q = h.face + (nb * 6 + (f ^ 1)) * 5;
                    for (int x = 0; x < 5; ++x) s[x] += hout[x] + q[x];
                }
            }
            for (int x = 0; x < 5; ++x) acc[x] += sg * (s[x] / double(nk));
            continue;
        }
        double hin[5] = {0, 0, 0, 0, 0};
        for (int k = 0; k < nk; ++k) {
            const int64_t nb = cell.nbr[f][k];
            double t[5];
            if (h.mask[nb] == 0) {
                sep_flux(h.flux + nb * kFluxRec, b, side ? 14 : 6, w, t);
            } else {
                const double *q = h.face + (nb * 6 + (f ^ 1)) * 5;  // leaving nb towards c
                for (int x = 0; x < 5; ++x) t[x] = q[x];
            }
            for (int x = 0; x < 5; ++x) hin[x] += t[x];
        }
        for (int x = 0; x < 5; ++x) acc[x] += sg * (hout[x] + hin[x] / double(nk));
    }
    const double dth = a.dt / hc;
    double U[5];
    for (int x = 0; x < 5; ++x) U[x] = a.mom[x * n + c] - dth * acc[x];
    for (int x = 0; x < 5; ++x) a.mom[x * n + c] = U[x];
    const double k2 = (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / U[0];
    if (!(U[0] > 0.0) || !(2.0 * U[4] - k2 > 0.0)) *a.flag = 1;
}

// After hybrid steps the f rows of fluid cells are stale and their state is
// the conserved moments U: copy U over what was recomputed from f.
__global__ __launch_bounds__(256) void k_fluid_moments(const uint8_t *mask, const double *mom, double *out,
                                                       int64_t n) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= n || mask[c]) return;
    for (int x = 0; x < 5; ++x) out[x * n + c] = mom[x * n + c];
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

template <typename F>
hipError_t labels_dispatch(const void *f, float *r, int64_t n, const VelGrid &g, hipStream_t st) {
    const F *p = static_cast<const F *>(f);
    const dim3 grid{unsigned(n), 1, 1};
    switch (g.nh) {
    case 2: hipLaunchKernelGGL((k_labels<F, 2, 64>), grid, dim3(64), 0, st, p, r, g); break;
    case 4: hipLaunchKernelGGL((k_labels<F, 4, 64>), grid, dim3(64), 0, st, p, r, g); break;
    case 6: hipLaunchKernelGGL((k_labels<F, 6, 256>), grid, dim3(256), 0, st, p, r, g); break;
    case 8: hipLaunchKernelGGL((k_labels<F, 8, 256>), grid, dim3(256), 0, st, p, r, g); break;
    case 12: hipLaunchKernelGGL((k_labels<F, 12, 576>), grid, dim3(576), 0, st, p, r, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename F>
hipError_t hybrid_dispatch(const StepArgs &a, const HybArgs &h, hipStream_t st) {
    const dim3 grid{unsigned(a.n_cells), 1, 1}, g256{unsigned((a.n_cells + 255) / 256), 1, 1};
    hipLaunchKernelGGL(k_fluid_state, g256, dim3(256), 0, st, a, h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define DVM_HYB(NH, T, W, FN)                                                                      \
    case NH:                                                                                       \
        hipLaunchKernelGGL((k_hybrid_rows<F, NH, T>), grid, dim3(T), 0, st, a, h);               \
        e = hipGetLastError();                                                                     \
        if (e != hipSuccess) return e;                                                             \
        hipLaunchKernelGGL((k_step_hybrid<F, NH, T, W, FN, true>), grid, dim3(T), 0, st, a, h); \
        break;
    switch (a.g.nh) {
        DVM_HYB(2, 64, 4, 0)
        DVM_HYB(4, 64, 5, 0)
        DVM_HYB(6, 256, 6, 0)
        DVM_HYB(8, 256, 5, 0)
        DVM_HYB(12, 192, 3, 1)
    default: return hipErrorInvalidValue;
    }
#undef DVM_HYB
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fluid_update, g256, dim3(256), 0, st, a, h);
    return hipGetLastError();
}

}  // namespace impl
}  // namespace dvm
