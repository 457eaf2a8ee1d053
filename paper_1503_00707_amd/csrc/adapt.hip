// adapt.hip -- on-device mesh adaptation.  Section 3.1 (step 4) rebuilds the
// cell order and the stencil each time the mesh changes; section 3.3 asks
// for everything to stay on the device.  Here the new leaf list (refinement,
// coarsening of complete sibling sets, then the 2:1 closure over faces, edges
// and corners of section 2.1), the per-cell face tables and the remapped
// state are all computed by kernels; only leaf counts cross to the host.
//
// Order without sorting.  Leaves are kept in Morton order on a fixed key
// lattice (level Lk, one below the finest level the adaptation can reach).
// The 8 children of a leaf, emitted in child order (x bit lowest), have
// ascending keys inside the parent's key range, and the parent of a complete
// sibling set takes the set's place: so emitting by an exclusive scan of
// per-leaf counts keeps the list sorted, and point location is a binary
// search over the keys.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <vector>

#include "solver_impl.h"

namespace dvm {
namespace {

struct Geo {
    int32_t base[3];
    int32_t per[3];
    int32_t Lk;       // key lattice level
    int64_t ext[3];   // lattice extent at Lk
};

__device__ __forceinline__ uint64_t spread(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
__device__ __forceinline__ uint64_t key_of(int64_t x, int64_t y, int64_t z) {
    return spread(uint64_t(x)) | (spread(uint64_t(y)) << 1) | (spread(uint64_t(z)) << 2);
}

struct Leaves {
    const uint8_t *level;
    const int32_t *ijk;
    const uint64_t *key;
    int64_t n;
};

__device__ __forceinline__ void corner(const Leaves &L, const Geo &g, int64_t t, int64_t c[3], int64_t &s) {
    const int sh = g.Lk - L.level[t];
    s = int64_t(1) << sh;
    for (int a = 0; a < 3; ++a) c[a] = int64_t(L.ijk[3 * t + a]) << sh;
}

// false if p leaves a non-periodic axis; periodic axes wrap
__device__ __forceinline__ bool wrap(const Geo &g, int64_t p[3]) {
    for (int a = 0; a < 3; ++a) {
        if (p[a] >= 0 && p[a] < g.ext[a]) continue;
        if (!g.per[a]) return false;
        p[a] = ((p[a] % g.ext[a]) + g.ext[a]) % g.ext[a];
    }
    return true;
}

// the leaf containing lattice point p: the last key <= key(p), if it covers p
__device__ int64_t find(const Leaves &L, const Geo &g, const int64_t p[3]) {
    const uint64_t k = key_of(p[0], p[1], p[2]);
    int64_t lo = 0, hi = L.n;  // first index with key > k
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (L.key[mid] <= k) lo = mid + 1;
        else hi = mid;
    }
    const int64_t t = lo - 1;
    if (t < 0) return -1;
    int64_t c[3], s;
    corner(L, g, t, c, s);
    for (int a = 0; a < 3; ++a)
        if (p[a] < c[a] || p[a] >= c[a] + s) return -1;
    return t;
}

__global__ __launch_bounds__(256) void k_keys(Leaves L, Geo g, uint64_t *key) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= L.n) return;
    int64_t c[3], s;
    corner(L, g, t, c, s);
    key[t] = key_of(c[0], c[1], c[2]);
}

__device__ __forceinline__ int child_index(const Leaves &L, int64_t t) {
    return (L.ijk[3 * t] & 1) | ((L.ijk[3 * t + 1] & 1) << 1) | ((L.ijk[3 * t + 2] & 1) << 2);
}

// leaves t0 .. t0+7 are the 8 children of one parent, in child order
__device__ bool sibling_set(const Leaves &L, int64_t t0) {
    if (t0 < 0 || t0 + 8 > L.n) return false;
    const int l = L.level[t0];
    if (l < 1) return false;
    for (int q = 0; q < 8; ++q) {
        const int64_t t = t0 + q;
        if (L.level[t] != l || child_index(L, t) != q) return false;
        for (int a = 0; a < 3; ++a)
            if ((L.ijk[3 * t + a] >> 1) != (L.ijk[3 * t0 + a] >> 1)) return false;
    }
    return true;
}

// leaves each old leaf becomes: 8 (refined), 0 or 1 (a coarsened sibling set
// is replaced by its parent at the first sibling's place), 1 (kept)
__global__ __launch_bounds__(256) void k_count(Leaves L, const int8_t *flags, int32_t *count) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= L.n) return;
    int c = 1;
    if (flags[t] > 0) {
        c = 8;
    } else if (flags[t] < 0) {
        const int64_t t0 = t - child_index(L, t);
        bool all = sibling_set(L, t0);
        for (int q = 0; q < 8 && all; ++q) all = flags[t0 + q] < 0;
        if (all) c = t == t0 ? 1 : 0;
    }
    count[t] = c;
}

// refinement of the leaves marked by the 2:1 closure
__global__ __launch_bounds__(256) void k_count_marked(int64_t n, const uint8_t *mark, int32_t *count) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t < n) count[t] = mark[t] ? 8 : 1;
}

__global__ __launch_bounds__(256) void k_emit(Leaves L, const int32_t *count, const int32_t *offset, uint8_t *lev_out,
                                              int32_t *ijk_out) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= L.n) return;
    const int c = count[t];
    const int64_t o = offset[t];
    const int l = L.level[t];
    const int32_t i = L.ijk[3 * t], j = L.ijk[3 * t + 1], k = L.ijk[3 * t + 2];
    if (c == 1) {
        // kept, or the parent of a coarsened set (emitted by its first child)
        const bool parent = count[t] == 1 && t + 1 < L.n && count[t + 1] == 0;
        lev_out[o] = uint8_t(parent ? l - 1 : l);
        ijk_out[3 * o] = parent ? i >> 1 : i;
        ijk_out[3 * o + 1] = parent ? j >> 1 : j;
        ijk_out[3 * o + 2] = parent ? k >> 1 : k;
    } else if (c == 8) {
        for (int q = 0; q < 8; ++q) {
            lev_out[o + q] = uint8_t(l + 1);
            ijk_out[3 * (o + q)] = 2 * i + (q & 1);
            ijk_out[3 * (o + q) + 1] = 2 * j + ((q >> 1) & 1);
            ijk_out[3 * (o + q) + 2] = 2 * k + ((q >> 2) & 1);
        }
    }
}

// leaves touched (face, edge or corner) by a leaf two or more levels finer:
// from each leaf the same-size region next to it in each of the 26
// directions lies inside any coarser leaf touching it there
__global__ __launch_bounds__(256) void k_violators(Leaves L, Geo g, uint8_t *mark, int *any) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= L.n) return;
    if (L.level[t] < 2) return;
    int64_t c[3], s;
    corner(L, g, t, c, s);
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                int64_t p[3] = {c[0] + dx * s, c[1] + dy * s, c[2] + dz * s};
                if (!wrap(g, p)) continue;
                const int64_t b = find(L, g, p);
                if (b >= 0 && L.level[b] + 2 <= L.level[t]) {
                    mark[b] = 1;
                    *any = 1;
                }
            }
}

// the per-cell face records of a leaf list without solids (the stencil of
// eq. 2): the same classification as the host builder; also whether the cell
// is regular (no FINER or WALL face: the step's reduced path) and the count
// of faces of each kind
__global__ __launch_bounds__(256) void k_tables(Leaves L, Geo g, const int32_t *bc, DevCell *out, int *bad,
                                                int32_t *regular, unsigned long long *n_faces) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= L.n) return;
    DevCell rec;
    memset(&rec, 0, sizeof rec);
    rec.level = L.level[t];
    int64_t c[3], s;
    corner(L, g, t, c, s);
    for (int f = 0; f < 6; ++f) {
        const int ax = f / 2, side = f % 2;
        for (int q = 0; q < 4; ++q) rec.nbr[f][q] = -1;
        int64_t p[3] = {c[0], c[1], c[2]};
        p[ax] += side ? s : -s;
        if (!wrap(g, p)) {
            const int b = bc[f];
            rec.type[f] = b == DVM_BC_INFLOW ? DVM_FACE_INFLOW : b == DVM_BC_OUTFLOW ? DVM_FACE_OUTFLOW : DVM_FACE_WALL;
            continue;
        }
        const int64_t b = find(L, g, p);
        if (b < 0) {
            *bad = 1;
            continue;
        }
        if (L.level[b] <= L.level[t]) {
            if (L.level[b] + 1 < L.level[t]) *bad = 1;
            rec.type[f] = L.level[b] == L.level[t] ? DVM_FACE_SAME : DVM_FACE_COARSER;
            rec.nbr[f][0] = int32_t(b);
            continue;
        }
        const int64_t hs = s / 2;
        const int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
        int64_t sub[4];
        for (int q = 0; q < 4; ++q) {
            int64_t r[3] = {p[0], p[1], p[2]};
            if (!side) r[ax] += hs;
            r[t1] += (q & 1) ? hs : 0;
            r[t2] += (q & 2) ? hs : 0;
            sub[q] = find(L, g, r);
            if (sub[q] < 0 || L.level[sub[q]] != L.level[t] + 1) *bad = 1;
        }
        // ascending leaf index (= key) order
        for (int x = 1; x < 4; ++x)
            for (int y = x; y > 0 && sub[y - 1] > sub[y]; --y) {
                const int64_t w = sub[y];
                sub[y] = sub[y - 1];
                sub[y - 1] = w;
            }
        rec.type[f] = DVM_FACE_FINER;
        for (int q = 0; q < 4; ++q) rec.nbr[f][q] = int32_t(sub[q]);
    }
    bool reg = true;
    for (int f = 0; f < 6; ++f) {
        if (rec.type[f] == DVM_FACE_WALL) rec.flags |= 1;
        reg &= rec.type[f] != DVM_FACE_FINER && rec.type[f] != DVM_FACE_WALL;
        atomicAdd(&n_faces[rec.type[f]], 1ull);
    }
    out[t] = rec;
    regular[t] = reg ? 1 : 0;
}

// the step's cell selection list: regular cells first, then the others, each
// in cell order (offset = exclusive scan of regular)
__global__ __launch_bounds__(256) void k_select(int64_t n, const int32_t *regular, const int32_t *offset,
                                                int64_t n_reg, uint32_t *sel) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= n) return;
    const int64_t o = offset[t];
    sel[regular[t] ? o : n_reg + (t - o)] = uint32_t(t);
}

// state of the new mesh: a new cell inside an old leaf (kept or refined)
// takes that leaf's row; a new cell covering several old leaves (coarsened)
// takes their volume-weighted mean, summed in FP64 in key order -- mass,
// momentum and energy are conserved.  One workgroup per new cell.
template <typename F>
__global__ __launch_bounds__(256) void k_remap(Leaves O, Leaves N, Geo g, const F *fo, F *fn, int64_t nv) {
    const int64_t t = blockIdx.x;
    int64_t c[3], s;
    corner(N, g, t, c, s);
    const int64_t a = find(O, g, c);
    if (a < 0) return;
    F *dst = fn + t * nv;
    if (O.level[a] <= N.level[t]) {
        const F *src = fo + a * nv;
        for (int64_t v = threadIdx.x; v < nv; v += 256) dst[v] = src[v];
        return;
    }
    // the old leaves inside: keys in [key, key + s^3)
    const uint64_t k_end = N.key[t] + uint64_t(s) * uint64_t(s) * uint64_t(s);
    int64_t e = a;
    while (e < O.n && O.key[e] < k_end) ++e;
    for (int64_t v = threadIdx.x; v < nv; v += 256) {
        double acc = 0.0;
        for (int64_t b = a; b < e; ++b) acc += ldexp(double(fo[b * nv + v]), -3 * (O.level[b] - N.level[t]));
        dst[v] = F(acc);
    }
}

int64_t blocks(int64_t n) { return (n + 255) / 256; }

}  // namespace
}  // namespace dvm

using namespace dvm;

namespace {

struct AdaptWs {
    // device scratch carved from the caller's workspace
    uint8_t *lev[2];
    int32_t *ijk[2];
    uint64_t *key;
    int32_t *count, *offset;
    uint8_t *mark;
    int *flag;
    void *scan_tmp;
    size_t scan_bytes;
};

size_t scan_temp_bytes(int64_t cap) {
    size_t b = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, b, static_cast<int32_t *>(nullptr),
                                           static_cast<int32_t *>(nullptr), int(cap));
    return b;
}

size_t carve(char *base, int64_t cap, AdaptWs *w) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + o : nullptr;
        o += align256(bytes);
        return p;
    };
    for (int k = 0; k < 2; ++k) {
        w->lev[k] = reinterpret_cast<uint8_t *>(take(size_t(cap)));
        w->ijk[k] = reinterpret_cast<int32_t *>(take(size_t(cap) * 12));
    }
    w->key = reinterpret_cast<uint64_t *>(take(size_t(cap) * 8));
    w->count = reinterpret_cast<int32_t *>(take(size_t(cap) * 4));
    w->offset = reinterpret_cast<int32_t *>(take(size_t(cap) * 4));
    w->mark = reinterpret_cast<uint8_t *>(take(size_t(cap)));
    w->flag = reinterpret_cast<int *>(take(256));
    w->scan_bytes = scan_temp_bytes(cap);
    w->scan_tmp = take(w->scan_bytes);
    return o;
}

Geo geo_of(const dvm_mesh *m, int Lk) {
    Geo g{};
    g.Lk = Lk;
    for (int a = 0; a < 3; ++a) {
        g.base[a] = m->base[a];
        g.per[a] = m->bc[2 * a] == DVM_BC_PERIODIC;
        g.ext[a] = int64_t(m->base[a]) << Lk;
    }
    return g;
}

// sum of count[0..n) and the exclusive offsets (synchronises)
int scan_counts(const AdaptWs &w, int64_t n, int64_t *total, hipStream_t st) {
    size_t tb = w.scan_bytes;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(w.scan_tmp, tb, w.count, w.offset, int(n), st);
    int32_t last_off = 0, last_cnt = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&last_off, w.offset + n - 1, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&last_cnt, w.count + n - 1, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "adapt scan");
    *total = int64_t(last_off) + last_cnt;
    return DVM_OK;
}

}  // namespace

extern "C" {

int dvm_adapt_workspace_bytes(int64_t max_leaves, size_t *bytes) {
    clear_error();
    if (!bytes || max_leaves < 1) return fail(DVM_ERR_ARG, "bad argument");
    if (max_leaves >= (int64_t(1) << 31)) return fail(DVM_ERR_UNSUPPORTED, "too many leaves");
    AdaptWs w{};
    *bytes = carve(nullptr, max_leaves, &w);
    return DVM_OK;
}

int dvm_adapt_leaves(const dvm_solver *s, const int8_t *flags, int64_t cap, uint8_t *level_out, int32_t *ijk_out,
                     int64_t *n_out, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!s || !flags || !level_out || !ijk_out || !n_out || !ws) return fail(DVM_ERR_ARG, "null argument");
    const dvm_mesh *m = s->m;
    if (int64_t(m->cells.size()) != m->n_leaves) return fail(DVM_ERR_UNSUPPORTED, "meshes with solid leaves");
    if (cap < m->n_leaves) return fail(DVM_ERR_ARG, "cap below the current leaf count");
    const int Lk = m->finest + 1;
    for (int a = 0; a < 3; ++a)
        if ((int64_t(m->base[a]) << Lk) >= (int64_t(1) << 21)) return fail(DVM_ERR_UNSUPPORTED, "domain too fine");
    AdaptWs w{};
    if (carve(nullptr, cap, &w) > ws_bytes) return fail(DVM_ERR_WORKSPACE, "workspace too small for %lld leaves",
                                                         (long long)cap);
    carve(static_cast<char *>(ws), cap, &w);
    hipStream_t st = S(stream);
    const Geo g = geo_of(m, Lk);
    // the current leaves (cell order = Morton order; no solids)
    int64_t n = m->n_leaves;
    {
        std::vector<uint8_t> lv(static_cast<size_t>(n));
        std::vector<int32_t> ij(static_cast<size_t>(3 * n));
        for (int64_t t = 0; t < n; ++t) {
            const Leaf &a = m->cells[size_t(t)];
            lv[size_t(t)] = a.level;
            ij[size_t(3 * t)] = a.i;
            ij[size_t(3 * t + 1)] = a.j;
            ij[size_t(3 * t + 2)] = a.k;
        }
        hipError_t e = hipMemcpyAsync(w.lev[0], lv.data(), size_t(n), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(w.ijk[0], ij.data(), size_t(12 * n), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // host arrays go out of scope
        if (e != hipSuccess) return hip_fail(e, "adapt upload");
    }
    int cur = 0;
    auto leaves = [&](int k, int64_t cnt) { return Leaves{w.lev[k], w.ijk[k], w.key, cnt}; };
    // refinement and coarsening as asked
    hipLaunchKernelGGL(k_keys, dim3(unsigned(blocks(n))), dim3(256), 0, st, leaves(cur, n), g, w.key);
    hipLaunchKernelGGL(k_count, dim3(unsigned(blocks(n))), dim3(256), 0, st, leaves(cur, n), flags, w.count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adapt count");
    int64_t total = 0;
    int rc = scan_counts(w, n, &total, st);
    if (rc) return rc;
    if (total > cap) {
        *n_out = total;
        return fail(DVM_ERR_WORKSPACE, "the adapted mesh has %lld leaves, cap %lld", (long long)total, (long long)cap);
    }
    hipLaunchKernelGGL(k_emit, dim3(unsigned(blocks(n))), dim3(256), 0, st, leaves(cur, n), w.count, w.offset,
                       w.lev[cur ^ 1], w.ijk[cur ^ 1]);
    cur ^= 1;
    n = total;
    // 2:1 closure: refine every leaf a finer leaf two levels down touches, until none
    for (int it = 0;; ++it) {
        hipLaunchKernelGGL(k_keys, dim3(unsigned(blocks(n))), dim3(256), 0, st, leaves(cur, n), g, w.key);
        e = hipMemsetAsync(w.mark, 0, size_t(n), st);
        if (e == hipSuccess) e = hipMemsetAsync(w.flag, 0, sizeof(int), st);
        if (e != hipSuccess) return hip_fail(e, "adapt closure");
        hipLaunchKernelGGL(k_violators, dim3(unsigned(blocks(n))), dim3(256), 0, st, leaves(cur, n), g, w.mark,
                           w.flag);
        int any = 0;
        e = hipMemcpyAsync(&any, w.flag, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "adapt closure");
        if (!any) break;
        if (it > 64) return fail(DVM_ERR_UNBALANCED, "2:1 closure did not converge");
        hipLaunchKernelGGL(k_count_marked, dim3(unsigned(blocks(n))), dim3(256), 0, st, n, w.mark, w.count);
        rc = scan_counts(w, n, &total, st);
        if (rc) return rc;
        if (total > cap) {
            *n_out = total;
            return fail(DVM_ERR_WORKSPACE, "the adapted mesh has %lld leaves, cap %lld", (long long)total,
                        (long long)cap);
        }
        hipLaunchKernelGGL(k_emit, dim3(unsigned(blocks(n))), dim3(256), 0, st, leaves(cur, n), w.count, w.offset,
                           w.lev[cur ^ 1], w.ijk[cur ^ 1]);
        cur ^= 1;
        n = total;
    }
    e = hipMemcpyAsync(level_out, w.lev[cur], size_t(n), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ijk_out, w.ijk[cur], size_t(12 * n), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "adapt output");
    *n_out = n;
    return DVM_OK;
}

int dvm_adapt_tables(dvm_solver *s, const uint8_t *level, const int32_t *ijk, void *ws, size_t ws_bytes,
                     void *stream) {
    clear_error();
    if (!s || !level || !ijk || !ws) return fail(DVM_ERR_ARG, "null argument");
    if (!s->tables) return fail(DVM_ERR_WORKSPACE, "solver not bound");
    if (!s->uploaded && !s->tables_pending) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    dvm_mesh *m = const_cast<dvm_mesh *>(s->m);
    if (int64_t(m->cells.size()) != m->n_leaves) return fail(DVM_ERR_UNSUPPORTED, "meshes with solid leaves");
    const int64_t n = s->n;
    AdaptWs w{};
    if (carve(nullptr, n, &w) > ws_bytes) return fail(DVM_ERR_WORKSPACE, "workspace too small");
    carve(static_cast<char *>(ws), n, &w);
    hipStream_t st = S(stream);
    const Geo g = geo_of(m, m->finest);
    // the 256-byte flag block: the error flag at 0, the boundary kinds at 16, face counts at 64
    int32_t *bc = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(w.flag) + 16);
    unsigned long long *nf = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(w.flag) + 64);
    hipError_t e = hipMemsetAsync(w.flag, 0, 256, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bc, m->bc, sizeof m->bc, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "adapt tables");
    const Leaves L{level, ijk, w.key, n};
    hipLaunchKernelGGL(k_keys, dim3(unsigned(blocks(n))), dim3(256), 0, st, L, g, w.key);
    hipLaunchKernelGGL(k_tables, dim3(unsigned(blocks(n))), dim3(256), 0, st, L, g, bc, s->tables, w.flag, w.count,
                       nf);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adapt tables");
    int64_t n_reg = 0;
    int rc = scan_counts(w, n, &n_reg, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_select, dim3(unsigned(blocks(n))), dim3(256), 0, st, n, w.count, w.offset, n_reg,
                       reinterpret_cast<uint32_t *>(s->ws + s->off_sel));
    int bad = 0;
    unsigned long long counts[6] = {0, 0, 0, 0, 0, 0};
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, w.flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(counts, nf, sizeof counts, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "adapt tables");
    if (bad) return fail(DVM_ERR_UNBALANCED, "the leaf list is not a 2:1-balanced partition");
    s->n_reg = n_reg;
    for (int f = 0; f < 6; ++f) m->n_faces[f] = int64_t(counts[f]);
    if (s->tables_pending) {
        s->tables_pending = false;
        s->uploaded = true;
    }
    return DVM_OK;
}

int dvm_adapt_mesh(const dvm_mesh *old, const uint8_t *level, const int32_t *ijk, int64_t n, dvm_mesh **out,
                   void *stream) {
    clear_error();
    if (!old || !level || !ijk || !out || n < 1) return fail(DVM_ERR_ARG, "bad argument");
    if (int64_t(old->cells.size()) != old->n_leaves) return fail(DVM_ERR_UNSUPPORTED, "meshes with solid leaves");
    if (n >= (int64_t(1) << 31)) return fail(DVM_ERR_UNSUPPORTED, "too many leaves");
    *out = nullptr;
    hipStream_t st = S(stream);
    std::vector<uint8_t> lv(static_cast<size_t>(n));
    std::vector<int32_t> ij(static_cast<size_t>(3 * n));
    hipError_t e = hipMemcpyAsync(lv.data(), level, size_t(n), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ij.data(), ijk, size_t(12 * n), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "adapt mesh");
    dvm_mesh *m = new (std::nothrow) dvm_mesh();
    if (!m) return fail(DVM_ERR_ARG, "out of host memory");
    for (int a = 0; a < 3; ++a) m->base[a] = old->base[a];
    for (int f = 0; f < 6; ++f) m->bc[f] = old->bc[f];
    m->h0 = old->h0;
    int L = 0;
    for (int64_t t = 0; t < n; ++t) L = std::max(L, int(lv[size_t(t)]));
    if (L > 20) {
        delete m;
        return fail(DVM_ERR_ARG, "level above 20");
    }
    m->cells.resize(size_t(n));
    for (int64_t t = 0; t < n; ++t) {
        Leaf &a = m->cells[size_t(t)];
        a.level = lv[size_t(t)];
        a.i = ij[size_t(3 * t)];
        a.j = ij[size_t(3 * t + 1)];
        a.k = ij[size_t(3 * t + 2)];
        a.input = t;
        a.solid = 0;
        const int sh = L - a.level;
        a.key = morton3(uint64_t(a.i) << sh, uint64_t(a.j) << sh, uint64_t(a.k) << sh);
    }
    m->finest = L;
    m->n_leaves = n;
    m->h_min = m->h0 / double(int64_t(1) << L);
    for (int f = 0; f < 6; ++f) m->n_faces[f] = 0;
    m->device_tables = true;
    *out = m;
    return DVM_OK;
}

int dvm_adapt_remap(const dvm_solver *from, dvm_solver *to, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!from || !to || !ws) return fail(DVM_ERR_ARG, "null argument");
    if (!from->uploaded || !to->uploaded) return fail(DVM_ERR_WORKSPACE, "both solvers must be uploaded");
    if (from->fp64 != to->fp64 || from->nv != to->nv || from->p.vmax[0] != to->p.vmax[0])
        return fail(DVM_ERR_ARG, "the solvers differ in precision or velocity grid");
    const dvm_mesh *a = from->m, *b = to->m;
    for (int x = 0; x < 3; ++x)
        if (a->base[x] != b->base[x] || a->h0 != b->h0) return fail(DVM_ERR_ARG, "the meshes cover different domains");
    if (from->hybrid_fluid) return fail(DVM_ERR_UNSUPPORTED, "fluid cells of a hybrid step hold no f");
    const int64_t na = from->n, nb = to->n;
    if (int64_t(a->cells.size()) != a->n_leaves || int64_t(b->cells.size()) != b->n_leaves)
        return fail(DVM_ERR_UNSUPPORTED, "meshes with solid leaves");
    const int Lk = std::max(a->finest, b->finest);
    for (int x = 0; x < 3; ++x)
        if ((int64_t(a->base[x]) << Lk) >= (int64_t(1) << 21)) return fail(DVM_ERR_UNSUPPORTED, "domain too fine");
    // both leaf lists and their keys in the workspace: [lev_a | ijk_a | key_a | lev_b | ijk_b | key_b]
    const size_t need = align256(size_t(na)) + align256(size_t(12 * na)) + align256(size_t(8 * na)) +
                        align256(size_t(nb)) + align256(size_t(12 * nb)) + align256(size_t(8 * nb));
    if (need > ws_bytes) return fail(DVM_ERR_WORKSPACE, "workspace too small");
    char *p = static_cast<char *>(ws);
    uint8_t *la = reinterpret_cast<uint8_t *>(p);
    int32_t *ia = reinterpret_cast<int32_t *>(p + align256(size_t(na)));
    uint64_t *ka = reinterpret_cast<uint64_t *>(p + align256(size_t(na)) + align256(size_t(12 * na)));
    char *q = p + align256(size_t(na)) + align256(size_t(12 * na)) + align256(size_t(8 * na));
    uint8_t *lb = reinterpret_cast<uint8_t *>(q);
    int32_t *ib = reinterpret_cast<int32_t *>(q + align256(size_t(nb)));
    uint64_t *kb = reinterpret_cast<uint64_t *>(q + align256(size_t(nb)) + align256(size_t(12 * nb)));
    hipStream_t st = S(stream);
    std::vector<uint8_t> lv;
    std::vector<int32_t> ij;
    auto upload = [&](const dvm_mesh *m, uint8_t *dl, int32_t *di) -> hipError_t {
        const int64_t n = int64_t(m->cells.size());
        lv.resize(size_t(n));
        ij.resize(size_t(3 * n));
        for (int64_t t = 0; t < n; ++t) {
            lv[size_t(t)] = m->cells[size_t(t)].level;
            ij[size_t(3 * t)] = m->cells[size_t(t)].i;
            ij[size_t(3 * t + 1)] = m->cells[size_t(t)].j;
            ij[size_t(3 * t + 2)] = m->cells[size_t(t)].k;
        }
        hipError_t e = hipMemcpyAsync(dl, lv.data(), size_t(n), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(di, ij.data(), size_t(12 * n), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        return e;
    };
    hipError_t e = upload(a, la, ia);
    if (e == hipSuccess) e = upload(b, lb, ib);
    if (e != hipSuccess) return hip_fail(e, "remap upload");
    const Geo g = geo_of(a, Lk);
    const Leaves A{la, ia, ka, na}, B{lb, ib, kb, nb};
    hipLaunchKernelGGL(k_keys, dim3(unsigned(blocks(na))), dim3(256), 0, st, A, g, ka);
    hipLaunchKernelGGL(k_keys, dim3(unsigned(blocks(nb))), dim3(256), 0, st, B, g, kb);
    // the internal velocity order is the same on both sides: remap rows as they are
    if (from->fp64)
        hipLaunchKernelGGL(k_remap<double>, dim3(unsigned(nb)), dim3(256), 0, st, A, B, g,
                           static_cast<const double *>(from->f[from->cur]), static_cast<double *>(to->f[to->cur]),
                           from->nv);
    else
        hipLaunchKernelGGL(k_remap<float>, dim3(unsigned(nb)), dim3(256), 0, st, A, B, g,
                           static_cast<const float *>(from->f[from->cur]), static_cast<float *>(to->f[to->cur]),
                           from->nv);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "remap");
    // the new buffer holds f itself: fresh records, masks and moments
    e = solver_state_replaced(to, st);
    return e == hipSuccess ? DVM_OK : hip_fail(e, "remap state");
}

}  // extern "C"
