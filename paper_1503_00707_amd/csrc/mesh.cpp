// mesh.cpp -- host mesh builder of the library: a linear octree (leaves as a
// sorted array of Morton keys) with point location by binary search.
//
// Section 2.1 of the paper fixes what is built: computations run on leaves
// only, the levels of direct and diagonal neighbours differ by at most one,
// and cells follow the Morton ("N-order") space-filling curve.  Section 3.1
// (step 4) asks for a per-cell stencil that is rebuilt when the mesh changes:
// here, 6 face records (kind + up to 4 neighbour cells).
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace dvm {

static thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}
void clear_error() { g_error.clear(); }

static inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
uint64_t morton3(uint64_t x, uint64_t y, uint64_t z) { return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2); }

namespace {

struct Linear {
    int32_t base[3];
    bool per[3];
    int L = 0;              // finest level
    int64_t ext[3];         // lattice extent at the finest level
    std::vector<Leaf> v;    // sorted by key

    int64_t span(const Leaf &a) const { return int64_t(1) << (L - a.level); }
    void corner(const Leaf &a, int64_t c[3]) const {
        int sh = L - a.level;
        c[0] = int64_t(a.i) << sh;
        c[1] = int64_t(a.j) << sh;
        c[2] = int64_t(a.k) << sh;
    }
    void rekey() {
        for (auto &a : v) {
            int64_t c[3];
            corner(a, c);
            a.key = morton3(c[0], c[1], c[2]);
        }
        std::sort(v.begin(), v.end(), [](const Leaf &a, const Leaf &b) { return a.key < b.key; });
    }
    // wrap a finest-lattice point; false if it leaves a non-periodic axis
    bool wrap(int64_t p[3]) const {
        for (int a = 0; a < 3; ++a) {
            if (p[a] >= 0 && p[a] < ext[a]) continue;
            if (!per[a]) return false;
            p[a] = ((p[a] % ext[a]) + ext[a]) % ext[a];
        }
        return true;
    }
    // index of the leaf containing lattice point p (already wrapped)
    int64_t find(const int64_t p[3]) const {
        uint64_t k = morton3(p[0], p[1], p[2]);
        auto it = std::upper_bound(v.begin(), v.end(), k, [](uint64_t x, const Leaf &a) { return x < a.key; });
        if (it == v.begin()) return -1;
        int64_t t = (it - v.begin()) - 1;
        int64_t c[3], s = span(v[t]);
        corner(v[t], c);
        for (int a = 0; a < 3; ++a)
            if (p[a] < c[a] || p[a] >= c[a] + s) return -1;
        return t;
    }
};

int load(const dvm_mesh_desc *d, Linear &T) {
    if (!d) return fail(DVM_ERR_ARG, "null mesh description");
    for (int a = 0; a < 3; ++a)
        if (d->base[a] < 1) return fail(DVM_ERR_ARG, "base[%d] = %d must be >= 1", a, d->base[a]);
    for (int f = 0; f < 6; ++f)
        if (d->bc[f] < DVM_BC_PERIODIC || d->bc[f] > DVM_BC_WALL) return fail(DVM_ERR_ARG, "bc[%d] invalid", f);
    for (int a = 0; a < 3; ++a) {
        bool lo = d->bc[2 * a] == DVM_BC_PERIODIC, hi = d->bc[2 * a + 1] == DVM_BC_PERIODIC;
        if (lo != hi) return fail(DVM_ERR_ARG, "axis %d: only one face periodic", a);
        T.per[a] = lo;
        T.base[a] = d->base[a];
    }
    if (!(d->h0 > 0)) return fail(DVM_ERR_ARG, "h0 must be > 0");
    if (d->n_leaves < 1 || !d->level || !d->ijk) return fail(DVM_ERR_ARG, "empty leaf list");
    T.v.resize(size_t(d->n_leaves));
    int L = 0;
    for (int64_t t = 0; t < d->n_leaves; ++t) {
        Leaf &a = T.v[size_t(t)];
        a.level = d->level[t];
        a.i = d->ijk[3 * t];
        a.j = d->ijk[3 * t + 1];
        a.k = d->ijk[3 * t + 2];
        a.input = t;
        a.solid = d->solid ? (d->solid[t] != 0) : 0;
        if (a.level > 20) return fail(DVM_ERR_ARG, "leaf %lld: level %d > 20", (long long)t, a.level);
        int64_t c[3] = {a.i, a.j, a.k};
        for (int x = 0; x < 3; ++x)
            if (c[x] < 0 || c[x] >= (int64_t(d->base[x]) << a.level))
                return fail(DVM_ERR_NOT_PARTITION, "leaf %lld lies outside the domain", (long long)t);
        L = std::max(L, int(a.level));
    }
    T.L = L;
    for (int a = 0; a < 3; ++a) {
        T.ext[a] = int64_t(d->base[a]) << L;
        if (T.ext[a] >= (int64_t(1) << 21)) return fail(DVM_ERR_ARG, "domain too fine for 63-bit Morton keys");
    }
    T.rekey();
    // exact partition: no two key ranges overlap and the volumes add up
    unsigned __int128 vol = 0;
    for (size_t t = 0; t < T.v.size(); ++t) {
        unsigned __int128 len = (unsigned __int128)1 << (3 * (L - T.v[t].level));
        vol += len;
        if (t + 1 < T.v.size() && (unsigned __int128)T.v[t].key + len > T.v[t + 1].key)
            return fail(DVM_ERR_NOT_PARTITION, "leaves %lld and %lld overlap", (long long)T.v[t].input,
                        (long long)T.v[t + 1].input);
    }
    unsigned __int128 full = (unsigned __int128)d->base[0] * d->base[1] * d->base[2] << (3 * L);
    if (vol != full) return fail(DVM_ERR_NOT_PARTITION, "leaves do not cover the domain");
    return DVM_OK;
}

// Leaves that a finer leaf two or more levels down touches (faces, edges,
// corners).  From each leaf a, the same-size region next to it in each of the
// 26 directions lies inside any coarser leaf that touches a there, so a point
// query at the region's corner finds it.
std::vector<char> coarse_violators(const Linear &T) {
    std::vector<char> mark(T.v.size(), 0);
    for (size_t t = 0; t < T.v.size(); ++t) {
        const Leaf &a = T.v[t];
        if (a.level < 2) continue;
        int64_t c[3], s = T.span(a);
        T.corner(a, c);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy && !dz) continue;
                    int64_t p[3] = {c[0] + dx * s, c[1] + dy * s, c[2] + dz * s};
                    if (!T.wrap(p)) continue;
                    int64_t b = T.find(p);
                    if (b >= 0 && T.v[size_t(b)].level + 2 <= a.level) mark[size_t(b)] = 1;
                }
    }
    return mark;
}

}  // namespace

static int build_tables(const Linear &T, dvm_mesh *m) {
    // fluid cells in Morton order, and leaf -> cell map
    std::vector<int64_t> cell_of(T.v.size(), -1);
    m->cells.clear();
    for (size_t t = 0; t < T.v.size(); ++t)
        if (!T.v[t].solid) {
            cell_of[t] = int64_t(m->cells.size());
            m->cells.push_back(T.v[t]);
        }
    if (m->cells.empty()) return fail(DVM_ERR_ARG, "no fluid leaf");
    if (m->cells.size() > size_t(INT32_MAX)) return fail(DVM_ERR_ARG, "too many cells for int32 tables");
    m->table.assign(m->cells.size(), DevCell{});
    std::memset(m->n_faces, 0, sizeof m->n_faces);
    int lmax = 0;
    for (size_t t = 0, c = 0; t < T.v.size(); ++t) {
        const Leaf &a = T.v[t];
        if (a.solid) continue;
        DevCell &rec = m->table[c++];
        std::memset(&rec, 0, sizeof rec);
        rec.level = a.level;
        lmax = std::max(lmax, int(a.level));
        int64_t corner[3], s = T.span(a);
        T.corner(a, corner);
        for (int f = 0; f < 6; ++f) {
            int ax = f / 2, side = f % 2;
            for (int q = 0; q < 4; ++q) rec.nbr[f][q] = -1;
            int64_t p[3] = {corner[0], corner[1], corner[2]};
            p[ax] += side ? s : -s;  // corner of the same-size region across the face
            if (!T.wrap(p)) {
                int bc = m->bc[f];
                rec.type[f] = bc == DVM_BC_INFLOW ? DVM_FACE_INFLOW : bc == DVM_BC_OUTFLOW ? DVM_FACE_OUTFLOW : DVM_FACE_WALL;
                continue;
            }
            int64_t b = T.find(p);
            if (b < 0) return fail(DVM_ERR_NOT_PARTITION, "no leaf across a face");
            const Leaf &nb = T.v[size_t(b)];
            if (nb.level <= a.level) {
                if (nb.level + 1 < a.level) return fail(DVM_ERR_UNBALANCED, "2:1 violated across a face");
                if (nb.solid) { rec.type[f] = DVM_FACE_WALL; continue; }
                rec.type[f] = nb.level == a.level ? DVM_FACE_SAME : DVM_FACE_COARSER;
                rec.nbr[f][0] = int32_t(cell_of[size_t(b)]);
                continue;
            }
            // subdivided region: the 4 half-size cubes touching the face
            int64_t hs = s / 2;
            int64_t sub[4];
            int n_solid = 0;
            int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
            for (int q = 0; q < 4; ++q) {
                int64_t r[3] = {p[0], p[1], p[2]};
                if (!side) r[ax] += hs;  // region below: its upper half touches the face
                r[t1] += (q & 1) ? hs : 0;
                r[t2] += (q & 2) ? hs : 0;
                int64_t e = T.find(r);
                if (e < 0 || T.v[size_t(e)].level != a.level + 1)
                    return fail(DVM_ERR_UNBALANCED, "2:1 violated across a face");
                sub[q] = e;
                n_solid += T.v[size_t(e)].solid;
            }
            if (n_solid == 4) { rec.type[f] = DVM_FACE_WALL; continue; }
            if (n_solid) return fail(DVM_ERR_UNSUPPORTED, "a coarse face is partly solid");
            std::sort(sub, sub + 4);  // leaf order is key order
            rec.type[f] = DVM_FACE_FINER;
            for (int q = 0; q < 4; ++q) rec.nbr[f][q] = int32_t(cell_of[size_t(sub[q])]);
        }
        for (int f = 0; f < 6; ++f) {
            m->n_faces[rec.type[f]]++;
            if (rec.type[f] == DVM_FACE_WALL) rec.flags |= 1;
        }
    }
    m->h_min = m->h0 / double(int64_t(1) << lmax);
    m->finest = T.L;
    m->n_leaves = int64_t(T.v.size());
    return DVM_OK;
}

}  // namespace dvm

using namespace dvm;

extern "C" {

const char *dvm_last_error(void) { return g_error.c_str(); }

int dvm_balance(const dvm_mesh_desc *d, int64_t cap, int64_t *n_out, uint8_t *level_out, int32_t *ijk_out) {
    clear_error();
    if (!n_out) return fail(DVM_ERR_ARG, "null n_out");
    try {
        Linear T;
        dvm_mesh_desc dd = *d;
        dd.solid = nullptr;
        int rc = load(&dd, T);
        if (rc) return rc;
        for (;;) {
            std::vector<char> mark = coarse_violators(T);
            size_t n_mark = size_t(std::count(mark.begin(), mark.end(), 1));
            if (!n_mark) break;
            std::vector<Leaf> next;
            next.reserve(T.v.size() + 7 * n_mark);
            for (size_t t = 0; t < T.v.size(); ++t) {
                if (!mark[t]) { next.push_back(T.v[t]); continue; }
                const Leaf &a = T.v[t];
                for (int c = 0; c < 8; ++c) {
                    Leaf ch = a;
                    ch.level = uint8_t(a.level + 1);
                    ch.i = 2 * a.i + (c & 1);
                    ch.j = 2 * a.j + ((c >> 1) & 1);
                    ch.k = 2 * a.k + ((c >> 2) & 1);
                    next.push_back(ch);
                }
            }
            T.v.swap(next);
            T.rekey();
        }
        *n_out = int64_t(T.v.size());
        if (int64_t(T.v.size()) > cap) return fail(DVM_ERR_WORKSPACE, "output holds %lld leaves, need %lld", (long long)cap, (long long)T.v.size());
        if (!level_out || !ijk_out) return fail(DVM_ERR_ARG, "null output");
        for (size_t t = 0; t < T.v.size(); ++t) {
            level_out[t] = T.v[t].level;
            ijk_out[3 * t] = T.v[t].i;
            ijk_out[3 * t + 1] = T.v[t].j;
            ijk_out[3 * t + 2] = T.v[t].k;
        }
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return fail(DVM_ERR_ARG, "out of host memory");
    }
}

int dvm_create_mesh(const dvm_mesh_desc *d, dvm_mesh **out) {
    clear_error();
    if (!out) return fail(DVM_ERR_ARG, "null out");
    *out = nullptr;
    try {
        Linear T;
        int rc = load(d, T);
        if (rc) return rc;
        std::vector<char> bad = coarse_violators(T);
        if (std::count(bad.begin(), bad.end(), 1)) return fail(DVM_ERR_UNBALANCED, "leaves violate the 2:1 rule");
        dvm_mesh *m = new dvm_mesh();
        for (int a = 0; a < 3; ++a) m->base[a] = d->base[a];
        for (int f = 0; f < 6; ++f) m->bc[f] = d->bc[f];
        m->h0 = d->h0;
        rc = build_tables(T, m);
        if (rc) { delete m; return rc; }
        *out = m;
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return fail(DVM_ERR_ARG, "out of host memory");
    }
}

int dvm_mesh_info(const dvm_mesh *m, dvm_mesh_info_t *out) {
    clear_error();
    if (!m || !out) return fail(DVM_ERR_ARG, "null argument");
    out->n_leaves = m->n_leaves;
    out->n_cells = int64_t(m->cells.size());
    out->max_level = m->finest;
    out->h_min = m->h_min;
    for (int f = 0; f < 6; ++f) out->n_faces[f] = m->n_faces[f];
    return DVM_OK;
}

int dvm_mesh_export(const dvm_mesh *m, int64_t *input, uint64_t *key, uint8_t *type, int32_t *nbr) {
    clear_error();
    if (!m) return fail(DVM_ERR_ARG, "null mesh");
    if (m->device_tables && (type || nbr))
        return fail(DVM_ERR_UNSUPPORTED, "this mesh's face tables live on the device (dvm_adapt_tables)");
    for (size_t c = 0; c < m->cells.size(); ++c) {
        if (input) input[c] = m->cells[c].input;
        if (key) key[c] = m->cells[c].key;
        for (int f = 0; f < 6; ++f) {
            if (type) type[6 * c + size_t(f)] = m->table[c].type[f];
            for (int q = 0; q < 4; ++q)
                if (nbr) nbr[24 * c + 4 * size_t(f) + size_t(q)] = m->table[c].nbr[f][q];
        }
    }
    return DVM_OK;
}

void dvm_destroy_mesh(dvm_mesh *m) { delete m; }

}  // extern "C"
