// korobov.cpp -- host side of the Boltzmann collision integral on Korobov
// lattice nodes (section 3.2, eqs. 3-6): the lattice generator, the per-node
// trial tables shared by every cell (eqs. 3-5: "the same for all points of
// [physical] space"), their export for tests.
//
// Tables.  For velocity node i (canonical index) and trial k = 0..p-1 of a
// p-point rank-1 Korobov lattice in 5 dimensions (generator a):
//   q_d = (k a^d + s_d(i)) mod p,  s_d(i) = (i + 1) c_d mod p,
//   c_d = (2654435761 mod p)(d + 1) mod p,                       d = 0..4,
//   partner node j_b = floor((q_b + 1/2) N_b / p)                 b = 0, 1, 2,
//   direction cos(theta) = 1 - 2 (q_3 + 1/2)/p,  phi = 2 pi (q_4 + 1/2)/p,
//   post-collision velocities c +- (|g|/2) n, c = (xi_i + xi_j)/2, g = xi_j - xi_i,
//   each in the node whose velocity cell holds it (none: the trial has no
//   gain term).  Node velocities are lo + (k + 1/2) d per axis, FP64.
// The device stores one 64-bit entry per (k, i) in its own velocity order
// (internal octant-major index), k-major so that the lanes of a wave (one node
// each) read consecutive entries: j | l << 16 | m << 32, with 0xFFFF for l
// and m when the trial has no gain term.  The weight V_box |g| / p is
// recomputed on the device from the nodes' velocities.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "solver_impl.h"

using namespace dvm;

namespace {

bool prime(int64_t p) {
    if (p < 2) return false;
    for (int64_t q = 2; q * q <= p; ++q)
        if (p % q == 0) return false;
    return true;
}

// P_2 figure of merit of the 5-dimensional lattice of generator a
double p2_merit(int64_t p, int64_t a) {
    const double two_pi2 = 2.0 * M_PI * M_PI;
    double sum = 0.0;
    for (int64_t k = 0; k < p; ++k) {
        double prod = 1.0;
        int64_t z = k;
        for (int d = 0; d < 5; ++d) {
            const double x = double(z) / double(p);
            prod *= 1.0 + two_pi2 * (x * x - x + 1.0 / 6.0);
            z = (z * a) % p;
        }
        sum += prod;
    }
    return sum / double(p) - 1.0;
}

// internal (octant-major) index of canonical node (kx, ky, kz)
int64_t internal_of(int nh, int kx, int ky, int kz) {
    const int sx = kx >= nh, sy = ky >= nh, sz = kz >= nh;
    const int ax = sx ? kx - nh : nh - 1 - kx, ay = sy ? ky - nh : nh - 1 - ky, az = sz ? kz - nh : nh - 1 - kz;
    const int64_t B = int64_t(nh) * nh * nh;
    return int64_t((sx << 2) | (sy << 1) | sz) * B + (int64_t(ax) * nh + ay) * nh + az;
}

}  // namespace

namespace dvm {

int64_t korobov_generator(int64_t p) {
    if (!prime(p) || p < 5 || p >= (int64_t(1) << 31)) return -1;
    int64_t best = -1;
    double best_v = 0.0;
    for (int64_t a = 2; a < p; ++a) {
        const double v = p2_merit(p, a);
        // a, -a, 1/a, -1/a (mod p) span the same lattice up to the order and
        // sign of coordinates: equal merit; the first of a tie wins
        if (best < 0 || v < best_v - 1e-9 * std::fabs(best_v)) {
            best = a;
            best_v = v;
        }
    }
    return best;
}

// canonical-index tables [i][k] (j, l, m; -1 for no gain term)
void korobov_tables(int n, double vmax, int64_t p, int64_t a, std::vector<int32_t> &J, std::vector<int32_t> &L,
                    std::vector<int32_t> &M) {
    const int64_t nv = int64_t(n) * n * n;
    J.assign(size_t(nv * p), 0);
    L.assign(size_t(nv * p), -1);
    M.assign(size_t(nv * p), -1);
    const double lo = -vmax, d = (vmax - lo) / n;
    std::vector<double> x(static_cast<size_t>(n));
    for (int k = 0; k < n; ++k) x[size_t(k)] = lo + (k + 0.5) * d;
    int64_t ap[5], c[5];
    ap[0] = 1;
    for (int e = 1; e < 5; ++e) ap[e] = ap[e - 1] * a % p;
    for (int e = 0; e < 5; ++e) c[e] = (int64_t(2654435761ll % p) * (e + 1)) % p;
    auto cell_of = [&](double v) -> int {
        const double t = std::floor((v - lo) / d);
        return (t < 0.0 || t >= double(n)) ? -1 : int(t);
    };
    for (int64_t i = 0; i < nv; ++i) {
        const int ix = int(i / (int64_t(n) * n)), iy = int((i / n) % n), iz = int(i % n);
        const double xi[3] = {x[size_t(ix)], x[size_t(iy)], x[size_t(iz)]};
        int64_t s[5];
        for (int e = 0; e < 5; ++e) s[e] = ((i + 1) % p) * c[e] % p;
        for (int64_t k = 0; k < p; ++k) {
            int64_t q[5];
            for (int e = 0; e < 5; ++e) q[e] = (k * ap[e] % p + s[e]) % p;
            int jb[3];
            for (int b = 0; b < 3; ++b) jb[b] = int(((2 * q[b] + 1) * n) / (2 * p));
            const double xs[3] = {x[size_t(jb[0])], x[size_t(jb[1])], x[size_t(jb[2])]};
            const double gx = xs[0] - xi[0], gy = xs[1] - xi[1], gz = xs[2] - xi[2];
            const double gg = std::sqrt(gx * gx + gy * gy + gz * gz);
            const double ct = 1.0 - 2.0 * ((double(q[3]) + 0.5) / double(p));
            const double st = std::sqrt(std::fmax(0.0, 1.0 - ct * ct));
            const double ph = 2.0 * M_PI * ((double(q[4]) + 0.5) / double(p));
            const double nn[3] = {st * std::cos(ph), st * std::sin(ph), ct};
            int l1[3], l2[3];
            bool ok = true;
            for (int b = 0; b < 3; ++b) {
                const double cb = 0.5 * (xi[b] + xs[b]);
                l1[b] = cell_of(cb + 0.5 * gg * nn[b]);
                l2[b] = cell_of(cb - 0.5 * gg * nn[b]);
                ok = ok && l1[b] >= 0 && l2[b] >= 0;
            }
            const size_t e = size_t(i * p + k);
            J[e] = int32_t((int64_t(jb[0]) * n + jb[1]) * n + jb[2]);
            if (ok) {
                L[e] = int32_t((int64_t(l1[0]) * n + l1[1]) * n + l1[2]);
                M[e] = int32_t((int64_t(l2[0]) * n + l2[1]) * n + l2[2]);
            }
        }
    }
}

// device form: [k][internal i], 64-bit entries
void korobov_device_table(int nh, const std::vector<int32_t> &J, const std::vector<int32_t> &L,
                          const std::vector<int32_t> &M, int64_t p, std::vector<uint64_t> &out) {
    const int n = 2 * nh;
    const int64_t nv = int64_t(n) * n * n;
    std::vector<int64_t> to_int(static_cast<size_t>(nv));
    for (int kx = 0; kx < n; ++kx)
        for (int ky = 0; ky < n; ++ky)
            for (int kz = 0; kz < n; ++kz) to_int[size_t((int64_t(kx) * n + ky) * n + kz)] = internal_of(nh, kx, ky, kz);
    out.assign(size_t(nv * p), 0);
    for (int64_t i = 0; i < nv; ++i)
        for (int64_t k = 0; k < p; ++k) {
            const size_t e = size_t(i * p + k);
            const uint64_t j = uint64_t(to_int[size_t(J[e])]);
            const uint64_t l = L[e] < 0 ? 0xFFFFu : uint64_t(to_int[size_t(L[e])]);
            const uint64_t m = M[e] < 0 ? 0xFFFFu : uint64_t(to_int[size_t(M[e])]);
            // |k_j - k_i|^2 in node units: |xi_j - xi_i| = dv sqrt(n) on the cubic grid
            const int64_t a = J[e], dx = a / (n * n) - i / (n * n), dy = (a / n) % n - (i / n) % n,
                          dz = a % n - i % n;
            const uint64_t g2 = uint64_t(dx * dx + dy * dy + dz * dz);
            out[size_t(k * nv + to_int[size_t(i)])] = j | (l << 16) | (m << 32) | (g2 << 48);
        }
}

}  // namespace dvm

extern "C" {

int dvm_korobov_generator(int64_t p, int64_t *a) {
    clear_error();
    if (!a) return fail(DVM_ERR_ARG, "null argument");
    *a = korobov_generator(p);
    if (*a < 0) return fail(DVM_ERR_ARG, "p = %lld must be a prime in [5, 2^31)", (long long)p);
    return DVM_OK;
}

int dvm_korobov_tables(int32_t nv, double vmax, int64_t p, int64_t a, int32_t *j, int32_t *l, int32_t *m) {
    clear_error();
    if (!j || !l || !m) return fail(DVM_ERR_ARG, "null argument");
    if (nv < 2 || nv > 256 || !(vmax > 0)) return fail(DVM_ERR_ARG, "bad velocity grid");
    if (!prime(p) || p < 5 || p >= (int64_t(1) << 31) || a < 1 || a >= p)
        return fail(DVM_ERR_ARG, "p must be a prime in [5, 2^31) and 1 <= a < p");
    std::vector<int32_t> J, L, M;
    korobov_tables(nv, vmax, p, a, J, L, M);
    std::copy(J.begin(), J.end(), j);
    std::copy(L.begin(), L.end(), l);
    std::copy(M.begin(), M.end(), m);
    return DVM_OK;
}

}  // extern "C"
