/*
 * dvm_oracle.c -- plain FP64 CPU oracle for the DVM-BGK step on an adaptive
 * octree (Zabelok, Arslanbekov & Kolobov, "Adaptive Kinetic-Fluid Solvers for
 * Heterogeneous Computing Architectures", arXiv:1503.00707).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library; it is deliberately slow and
 * written to be checked against the paper by eye:
 *
 *   mesh      -- pointer-based recursive octree per root cube (forest of trees,
 *                section 2.1 and 2.2), 2:1 balance over direct and diagonal
 *                neighbours (section 2.1), Morton ("N-order") leaf order
 *                (section 2.1), face classification by tree point location.
 *   transport -- finite-volume first-order upwind, explicit Euler: eq. (2) of
 *                section 3.1, written in flux form over leaf faces; an optional
 *                minmod-MUSCL face reconstruction (the paper is silent on it;
 *                the reading is stated at or_muscl_sigma()).
 *   collision -- BGK relaxation (section 4, the BGK form) toward a discrete
 *                Maxwellian corrected by the polynomial P of eq. (6) so that
 *                mass, momentum and energy are conserved (section 3.2); the
 *                5x5 system is solved by Gauss elimination (section 3.2).
 *                Or the Boltzmann collision integral of hard spheres on
 *                Korobov lattice nodes, eqs. (3)-(6) of section 3.2, with the
 *                same conservative correction (see or_korobov_tables()).
 *                Or the lattice Boltzmann BGK collision of section 4 on the
 *                D3Q19 / D3Q27 subsets of a 3x3x3 velocity grid.
 *
 * Everything is FP64.  f is stored cell-major in canonical velocity order
 * i = (kx*Ny + ky)*Nz + kz, cells in Morton order.  OpenMP parallelises the
 * loop over cells only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_UNBALANCED (-2)
#define OR_ERR_NOT_PARTITION (-3)
#define OR_ERR_NONPHYSICAL (-5)
#define OR_ERR_UNSUPPORTED (-7)

/* domain boundary kinds, per domain face (-x,+x,-y,+y,-z,+z) */
#define OR_BC_PERIODIC 0
#define OR_BC_INFLOW 1
#define OR_BC_OUTFLOW 2
#define OR_BC_WALL 3

/* face kinds in the neighbour table */
#define OR_FACE_SAME 0
#define OR_FACE_COARSER 1
#define OR_FACE_FINER 2
#define OR_FACE_INFLOW 3
#define OR_FACE_OUTFLOW 4
#define OR_FACE_WALL 5

/* ------------------------------------------------------------------------ */
/* Octree forest                                                            */
/* ------------------------------------------------------------------------ */

typedef struct or_node {
    struct or_node *child[8]; /* child c = cx + 2*cy + 4*cz; all NULL for a leaf */
    int level;
    int64_t i, j, k;          /* integer coordinates at this node's level */
    int is_leaf;              /* 1 once the node is a leaf of the partition */
    int solid;                /* leaf inside a solid body */
    int64_t cell;             /* index among fluid leaves (Morton rank), -1 else */
    int64_t input;            /* index in the caller's leaf list, -1 else */
} or_node;

typedef struct {
    int n[3];         /* root cubes per axis */
    int periodic[3];
    or_node **roots;  /* n[0]*n[1]*n[2], index (ri*n1 + rj)*n2 + rk */
} or_forest;

static or_node *node_new(int level, int64_t i, int64_t j, int64_t k) {
    or_node *p = (or_node *)calloc(1, sizeof(or_node));
    p->level = level;
    p->i = i; p->j = j; p->k = k;
    p->cell = -1;
    p->input = -1;
    return p;
}

static void node_free(or_node *p) {
    if (!p) return;
    for (int c = 0; c < 8; ++c) node_free(p->child[c]);
    free(p);
}

static void forest_free(or_forest *F) {
    if (!F) return;
    if (F->roots) {
        for (int r = 0; r < F->n[0] * F->n[1] * F->n[2]; ++r) node_free(F->roots[r]);
        free(F->roots);
    }
    free(F);
}

static or_forest *forest_new(const int n[3], const int periodic[3]) {
    or_forest *F = (or_forest *)calloc(1, sizeof(or_forest));
    for (int a = 0; a < 3; ++a) { F->n[a] = n[a]; F->periodic[a] = periodic[a]; }
    F->roots = (or_node **)calloc((size_t)n[0] * n[1] * n[2], sizeof(or_node *));
    for (int ri = 0; ri < n[0]; ++ri)
        for (int rj = 0; rj < n[1]; ++rj)
            for (int rk = 0; rk < n[2]; ++rk)
                F->roots[(ri * n[1] + rj) * n[2] + rk] = node_new(0, ri, rj, rk);
    return F;
}

static void node_split(or_node *p) {
    for (int c = 0; c < 8; ++c) {
        int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        p->child[c] = node_new(p->level + 1, 2 * p->i + cx, 2 * p->j + cy, 2 * p->k + cz);
    }
}

/* Insert one leaf by walking down from its root cube, creating children on
 * the way.  Returns 0, or OR_ERR_NOT_PARTITION on overlap. */
static int forest_insert(or_forest *F, int level, int64_t i, int64_t j, int64_t k, int64_t input) {
    if (level < 0 || level > 20) return OR_ERR_ARG;
    int64_t ri = i >> level, rj = j >> level, rk = k >> level;
    if (i < 0 || j < 0 || k < 0 || ri >= F->n[0] || rj >= F->n[1] || rk >= F->n[2]) return OR_ERR_ARG;
    or_node *p = F->roots[(ri * F->n[1] + rj) * F->n[2] + rk];
    for (int l = 1; l <= level; ++l) {
        if (p->is_leaf) return OR_ERR_NOT_PARTITION; /* an ancestor is already a leaf */
        if (!p->child[0]) node_split(p);
        int sh = level - l;
        int c = (int)((i >> sh) & 1) + 2 * (int)((j >> sh) & 1) + 4 * (int)((k >> sh) & 1);
        p = p->child[c];
    }
    if (p->is_leaf || p->child[0]) return OR_ERR_NOT_PARTITION; /* duplicate, or covers finer leaves */
    p->is_leaf = 1;
    p->input = input;
    return OR_OK;
}

/* every node must be a leaf or have 8 children that are (recursively) covered */
static int node_covered(const or_node *p) {
    if (p->is_leaf) return 1;
    if (!p->child[0]) return 0;
    for (int c = 0; c < 8; ++c)
        if (!node_covered(p->child[c])) return 0;
    return 1;
}

/* Locate the node covering cell (i,j,k) of the lattice at `level`.  Returns
 * the node at that level if the tree reaches it, otherwise the leaf that
 * contains it.  Periodic axes wrap; a position outside a non-periodic axis
 * returns NULL. */
static or_node *forest_locate(const or_forest *F, int level, int64_t i, int64_t j, int64_t k) {
    int64_t ext[3] = {(int64_t)F->n[0] << level, (int64_t)F->n[1] << level, (int64_t)F->n[2] << level};
    int64_t c[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (c[a] < 0 || c[a] >= ext[a]) {
            if (!F->periodic[a]) return NULL;
            c[a] = ((c[a] % ext[a]) + ext[a]) % ext[a];
        }
    }
    or_node *p = F->roots[((c[0] >> level) * F->n[1] + (c[1] >> level)) * F->n[2] + (c[2] >> level)];
    for (int l = 1; l <= level; ++l) {
        if (!p->child[0]) return p;
        int sh = level - l;
        int ch = (int)((c[0] >> sh) & 1) + 2 * (int)((c[1] >> sh) & 1) + 4 * (int)((c[2] >> sh) & 1);
        p = p->child[ch];
    }
    return p;
}

/* collect the leaves (any order) */
typedef struct { or_node **v; int64_t n, cap; } node_list;
static void list_push(node_list *L, or_node *p) {
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->v = (or_node **)realloc(L->v, (size_t)L->cap * sizeof(or_node *));
    }
    L->v[L->n++] = p;
}
static void collect_leaves(or_node *p, node_list *L) {
    if (p->is_leaf) { list_push(L, p); return; }
    for (int c = 0; c < 8; ++c)
        if (p->child[c]) collect_leaves(p->child[c], L);
}
static void forest_leaves(const or_forest *F, node_list *L) {
    for (int r = 0; r < F->n[0] * F->n[1] * F->n[2]; ++r) collect_leaves(F->roots[r], L);
}

/* 2:1 rule over direct and diagonal neighbours (section 2.1): leaf p violates
 * it when a leaf two or more levels finer touches it across a face, an edge or
 * a corner.  Such a leaf exists iff, in the same-size region next to p, the
 * tree has a node at p's level+1 that touches p and is itself subdivided. */
static int leaf_violates(const or_forest *F, const or_node *p) {
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                if (!dx && !dy && !dz) continue;
                or_node *q = forest_locate(F, p->level, p->i + dx, p->j + dy, p->k + dz);
                if (!q || q->level < p->level || !q->child[0]) continue;
                for (int c = 0; c < 8; ++c) {
                    int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
                    /* the child touches p iff it lies on the side facing p */
                    if (dx && cx != (dx < 0)) continue;
                    if (dy && cy != (dy < 0)) continue;
                    if (dz && cz != (dz < 0)) continue;
                    if (q->child[c]->child[0]) return 1;
                }
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Morton key on the finest lattice (section 2.1, "N-order")                */
/* ------------------------------------------------------------------------ */

static uint64_t morton_key(const or_node *p, int finest) {
    int sh = finest - p->level;
    uint64_t x = (uint64_t)p->i << sh, y = (uint64_t)p->j << sh, z = (uint64_t)p->k << sh;
    uint64_t key = 0;
    for (int b = 0; b < 21; ++b) {
        key |= ((x >> b) & 1ull) << (3 * b);
        key |= ((y >> b) & 1ull) << (3 * b + 1);
        key |= ((z >> b) & 1ull) << (3 * b + 2);
    }
    return key;
}

static int g_sort_finest; /* qsort has no context argument */
static int cmp_node_key(const void *a, const void *b) {
    uint64_t ka = morton_key(*(or_node *const *)a, g_sort_finest);
    uint64_t kb = morton_key(*(or_node *const *)b, g_sort_finest);
    return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

static int list_finest(const node_list *L) {
    int m = 0;
    for (int64_t t = 0; t < L->n; ++t)
        if (L->v[t]->level > m) m = L->v[t]->level;
    return m;
}

/* build a forest from a leaf list, checking it is a partition */
static int forest_from_leaves(const int n[3], const int periodic[3], int64_t n_leaves,
                              const uint8_t *level, const int32_t *ijk, or_forest **out) {
    or_forest *F = forest_new(n, periodic);
    for (int64_t t = 0; t < n_leaves; ++t) {
        int rc = forest_insert(F, level[t], ijk[3 * t], ijk[3 * t + 1], ijk[3 * t + 2], t);
        if (rc) { forest_free(F); return rc; }
    }
    for (int r = 0; r < n[0] * n[1] * n[2]; ++r)
        if (!node_covered(F->roots[r])) { forest_free(F); return OR_ERR_NOT_PARTITION; }
    *out = F;
    return OR_OK;
}

/*
 * or_balance: refine the given partition until the 2:1 rule holds over faces,
 * edges and corners (section 2.1); returns the leaves in Morton order.
 * `cap` is the capacity of the output arrays; *n_out is set even when it is
 * too small (then OR_ERR_ARG is returned and nothing is written).
 */
int or_balance(const int n[3], const int periodic[3], int64_t n_leaves, const uint8_t *level,
               const int32_t *ijk, int64_t cap, int64_t *n_out, uint8_t *level_out, int32_t *ijk_out) {
    or_forest *F;
    int rc = forest_from_leaves(n, periodic, n_leaves, level, ijk, &F);
    if (rc) return rc;
    for (;;) {
        node_list L = {0};
        forest_leaves(F, &L);
        int64_t n_split = 0;
        /* mark first, then split, so that one sweep sees one consistent tree */
        char *mark = (char *)calloc((size_t)L.n, 1);
        for (int64_t t = 0; t < L.n; ++t)
            if (leaf_violates(F, L.v[t])) { mark[t] = 1; ++n_split; }
        for (int64_t t = 0; t < L.n; ++t)
            if (mark[t]) {
                or_node *p = L.v[t];
                p->is_leaf = 0;
                node_split(p);
                for (int c = 0; c < 8; ++c) p->child[c]->is_leaf = 1;
            }
        free(mark);
        free(L.v);
        if (!n_split) break;
    }
    node_list L = {0};
    forest_leaves(F, &L);
    g_sort_finest = list_finest(&L);
    qsort(L.v, (size_t)L.n, sizeof(or_node *), cmp_node_key);
    *n_out = L.n;
    if (L.n > cap) { free(L.v); forest_free(F); return OR_ERR_ARG; }
    for (int64_t t = 0; t < L.n; ++t) {
        level_out[t] = (uint8_t)L.v[t]->level;
        ijk_out[3 * t] = (int32_t)L.v[t]->i;
        ijk_out[3 * t + 1] = (int32_t)L.v[t]->j;
        ijk_out[3 * t + 2] = (int32_t)L.v[t]->k;
    }
    free(L.v);
    forest_free(F);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Mesh: fluid leaves in Morton order and their face tables                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    or_forest *F;
    double h0;
    int bc[6];
    int64_t n_cells;      /* fluid leaves */
    int64_t n_leaves;     /* all leaves */
    int finest;
    or_node **cell;       /* fluid leaves in Morton order */
    uint8_t *type;        /* [n_cells][6] */
    int32_t *nbr;         /* [n_cells][6][4], -1 padding */
} or_mesh;

static int bc_face_kind(int bc) {
    switch (bc) {
    case OR_BC_INFLOW: return OR_FACE_INFLOW;
    case OR_BC_OUTFLOW: return OR_FACE_OUTFLOW;
    case OR_BC_WALL: return OR_FACE_WALL;
    default: return -1;
    }
}

void or_mesh_free(or_mesh *m) {
    if (!m) return;
    forest_free(m->F);
    free(m->cell);
    free(m->type);
    free(m->nbr);
    free(m);
}

/*
 * or_mesh_new: build the mesh from a leaf list that must be an exact, 2:1
 * balanced partition of the root cubes.  bc[6] gives the domain faces in the
 * order -x,+x,-y,+y,-z,+z; both faces of an axis are PERIODIC or neither is.
 * solid (may be NULL) flags leaves inside a body; a face between a fluid and a
 * solid leaf is a WALL face.
 */
int or_mesh_new(const int n[3], double h0, const int bc[6], int64_t n_leaves, const uint8_t *level,
                const int32_t *ijk, const uint8_t *solid, or_mesh **out) {
    int periodic[3];
    for (int a = 0; a < 3; ++a) {
        int lo = bc[2 * a] == OR_BC_PERIODIC, hi = bc[2 * a + 1] == OR_BC_PERIODIC;
        if (lo != hi) return OR_ERR_ARG;
        periodic[a] = lo;
    }
    or_forest *F;
    int rc = forest_from_leaves(n, periodic, n_leaves, level, ijk, &F);
    if (rc) return rc;
    node_list L = {0};
    forest_leaves(F, &L);
    for (int64_t t = 0; t < L.n; ++t)
        if (leaf_violates(F, L.v[t])) { free(L.v); forest_free(F); return OR_ERR_UNBALANCED; }
    g_sort_finest = list_finest(&L);
    qsort(L.v, (size_t)L.n, sizeof(or_node *), cmp_node_key);

    or_mesh *m = (or_mesh *)calloc(1, sizeof(or_mesh));
    m->F = F;
    m->h0 = h0;
    for (int f = 0; f < 6; ++f) m->bc[f] = bc[f];
    m->finest = g_sort_finest;
    m->n_leaves = L.n;
    m->cell = (or_node **)malloc((size_t)L.n * sizeof(or_node *));
    int64_t nc = 0;
    for (int64_t t = 0; t < L.n; ++t) {
        or_node *p = L.v[t];
        p->solid = solid ? (solid[p->input] != 0) : 0;
        if (!p->solid) { p->cell = nc; m->cell[nc++] = p; }
    }
    free(L.v);
    m->n_cells = nc;
    m->type = (uint8_t *)malloc((size_t)nc * 6);
    m->nbr = (int32_t *)malloc((size_t)nc * 24 * sizeof(int32_t));

    for (int64_t c = 0; c < nc; ++c) {
        or_node *p = m->cell[c];
        for (int f = 0; f < 6; ++f) {
            int axis = f / 2, side = f % 2; /* side 0: -, 1: + */
            int64_t d[3] = {0, 0, 0};
            d[axis] = side ? 1 : -1;
            uint8_t *ty = &m->type[c * 6 + f];
            int32_t *nb = &m->nbr[(c * 6 + f) * 4];
            nb[0] = nb[1] = nb[2] = nb[3] = -1;
            or_node *q = forest_locate(F, p->level, p->i + d[0], p->j + d[1], p->k + d[2]);
            if (!q) { /* outside a non-periodic axis: domain boundary */
                *ty = (uint8_t)bc_face_kind(bc[f]);
                continue;
            }
            if (q->is_leaf) {
                if (q->level != p->level && q->level != p->level - 1) { or_mesh_free(m); return OR_ERR_UNBALANCED; }
                if (q->solid) { *ty = OR_FACE_WALL; continue; }
                *ty = q->level == p->level ? OR_FACE_SAME : OR_FACE_COARSER;
                nb[0] = (int32_t)q->cell;
                continue;
            }
            /* the same-size region is subdivided: its 4 children on the side facing p */
            or_node *sub[4];
            int ns = 0, n_solid = 0;
            for (int ch = 0; ch < 8; ++ch) {
                int cc[3] = {ch & 1, (ch >> 1) & 1, (ch >> 2) & 1};
                if (cc[axis] != (side ? 0 : 1)) continue;
                or_node *s = q->child[ch];
                if (!s->is_leaf) { or_mesh_free(m); return OR_ERR_UNBALANCED; }
                sub[ns++] = s;
                n_solid += s->solid;
            }
            if (n_solid == 4) { *ty = OR_FACE_WALL; continue; }
            if (n_solid) { or_mesh_free(m); return OR_ERR_UNSUPPORTED; } /* partly solid coarse face */
            /* ascending Morton key (cell index is the Morton rank among fluid leaves) */
            for (int a = 0; a < 4; ++a)
                for (int b = a + 1; b < 4; ++b)
                    if (sub[b]->cell < sub[a]->cell) { or_node *t = sub[a]; sub[a] = sub[b]; sub[b] = t; }
            *ty = OR_FACE_FINER;
            for (int s = 0; s < 4; ++s) nb[s] = (int32_t)sub[s]->cell;
        }
    }
    *out = m;
    return OR_OK;
}

int64_t or_mesh_n_cells(const or_mesh *m) { return m->n_cells; }
int64_t or_mesh_n_leaves(const or_mesh *m) { return m->n_leaves; }

/* per fluid cell: Morton key, input index, level, ijk; face kinds and neighbours */
void or_mesh_export(const or_mesh *m, uint64_t *key, int64_t *input, uint8_t *level, int32_t *ijk,
                    uint8_t *type, int32_t *nbr) {
    for (int64_t c = 0; c < m->n_cells; ++c) {
        const or_node *p = m->cell[c];
        if (key) key[c] = morton_key(p, m->finest);
        if (input) input[c] = p->input;
        if (level) level[c] = (uint8_t)p->level;
        if (ijk) { ijk[3 * c] = (int32_t)p->i; ijk[3 * c + 1] = (int32_t)p->j; ijk[3 * c + 2] = (int32_t)p->k; }
    }
    if (type) memcpy(type, m->type, (size_t)m->n_cells * 6);
    if (nbr) memcpy(nbr, m->nbr, (size_t)m->n_cells * 24 * sizeof(int32_t));
}

static double cell_h(const or_mesh *m, int64_t c) { return m->h0 / (double)(1ll << m->cell[c]->level); }

/* ------------------------------------------------------------------------ */
/* Velocity grid (section 3: f at cell centres of a uniform Cartesian grid)  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n[3];
    double lo[3], hi[3];
    double d[3];  /* spacing per axis */
    double w;     /* cell volume in velocity space */
    int64_t nv;
    double *xi[3]; /* per-axis nodes */
} or_vgrid;

static void vgrid_init(or_vgrid *g, const int n[3], const double lo[3], const double hi[3]) {
    g->nv = 1;
    g->w = 1.0;
    for (int a = 0; a < 3; ++a) {
        g->n[a] = n[a];
        g->lo[a] = lo[a];
        g->hi[a] = hi[a];
        g->d[a] = (hi[a] - lo[a]) / n[a];
        g->w *= g->d[a];
        g->nv *= n[a];
        g->xi[a] = (double *)malloc((size_t)n[a] * sizeof(double));
        for (int k = 0; k < n[a]; ++k) g->xi[a][k] = lo[a] + (k + 0.5) * g->d[a];
    }
}
static void vgrid_free(or_vgrid *g) {
    for (int a = 0; a < 3; ++a) free(g->xi[a]);
}
/* velocity components of canonical index v */
static void vgrid_xi(const or_vgrid *g, int64_t v, double xi[3]) {
    int kz = (int)(v % g->n[2]);
    int ky = (int)((v / g->n[2]) % g->n[1]);
    int kx = (int)(v / ((int64_t)g->n[1] * g->n[2]));
    xi[0] = g->xi[0][kx];
    xi[1] = g->xi[1][ky];
    xi[2] = g->xi[2][kz];
}

/* ------------------------------------------------------------------------ */
/* Moments, Maxwellian and its conservative correction                      */
/* ------------------------------------------------------------------------ */

/* conserved moments (rho, rho*u, E) = w * sum_i (1, xi_i, |xi_i|^2/2) f_i */
static void moments_of(const or_vgrid *g, const double *f, double mom[5]) {
    double s[5] = {0, 0, 0, 0, 0};
    for (int64_t v = 0; v < g->nv; ++v) {
        double xi[3];
        vgrid_xi(g, v, xi);
        s[0] += f[v];
        s[1] += xi[0] * f[v];
        s[2] += xi[1] * f[v];
        s[3] += xi[2] * f[v];
        s[4] += 0.5 * (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]) * f[v];
    }
    for (int a = 0; a < 5; ++a) mom[a] = g->w * s[a];
}

/* rho, u, T from conserved moments; gas constant 1 (non-dimensional, eq. 1) */
static int primitive_of(const double mom[5], double *rho, double u[3], double *T) {
    *rho = mom[0];
    if (!(*rho > 0.0)) return OR_ERR_NONPHYSICAL;
    for (int a = 0; a < 3; ++a) u[a] = mom[1 + a] / *rho;
    *T = (2.0 * mom[4] / *rho - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / 3.0;
    if (!(*T > 0.0)) return OR_ERR_NONPHYSICAL;
    return OR_OK;
}

/* Gauss elimination with partial pivoting on an n x n system (section 3.2) */
static int gauss_solve(int n, double *A, double *b, double *x) {
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
        if (A[piv * n + col] == 0.0) return OR_ERR_NONPHYSICAL;
        if (piv != col) {
            for (int c = 0; c < n; ++c) { double t = A[col * n + c]; A[col * n + c] = A[piv * n + c]; A[piv * n + c] = t; }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            double q = A[r * n + col] / A[col * n + col];
            for (int c = col; c < n; ++c) A[r * n + c] -= q * A[col * n + c];
            b[r] -= q * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c) s -= A[r * n + c] * x[c];
        x[r] = s / A[r * n + r];
    }
    return OR_OK;
}

/*
 * Discrete Maxwellian corrected so that its discrete moments equal `target`
 * (rho, rho*u, E).  The raw Maxwellian M_i = rho (2 pi T)^(-3/2)
 * exp(-|xi_i - u|^2 / 2T) is multiplied by the polynomial of eq. (6),
 * P = 1 + d0 + dx xi_x + dy xi_y + dz xi_z + d2 |xi|^2, whose five
 * coefficients solve the five conservation equations
 *   sum_b d_b w sum_i psi_a psi_b M_i = target'_a - w sum_i psi_a M_i,
 * psi = (1, xi_x, xi_y, xi_z, |xi|^2) and target' the psi-moments of target.
 */
static int corrected_maxwellian(const or_vgrid *g, const double target[5], double *out) {
    double rho, u[3], T;
    int rc = primitive_of(target, &rho, u, &T);
    if (rc) return rc;
    double C = rho * pow(2.0 * M_PI * T, -1.5);
    double G[25], r[5], tpsi[5] = {target[0], target[1], target[2], target[3], 2.0 * target[4]};
    double sM[5] = {0, 0, 0, 0, 0};
    memset(G, 0, sizeof G);
    for (int64_t v = 0; v < g->nv; ++v) {
        double xi[3];
        vgrid_xi(g, v, xi);
        double dx = xi[0] - u[0], dy = xi[1] - u[1], dz = xi[2] - u[2];
        double M = C * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * T));
        double psi[5] = {1.0, xi[0], xi[1], xi[2], xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]};
        for (int a = 0; a < 5; ++a) {
            sM[a] += psi[a] * M;
            for (int b = 0; b < 5; ++b) G[a * 5 + b] += psi[a] * psi[b] * M;
        }
        out[v] = M;
    }
    for (int a = 0; a < 5; ++a) {
        r[a] = tpsi[a] - g->w * sM[a];
        for (int b = 0; b < 5; ++b) G[a * 5 + b] *= g->w;
    }
    double d[5];
    rc = gauss_solve(5, G, r, d);
    if (rc) return rc;
    for (int64_t v = 0; v < g->nv; ++v) {
        double xi[3];
        vgrid_xi(g, v, xi);
        double P = 1.0 + d[0] + d[1] * xi[0] + d[2] * xi[1] + d[3] * xi[2] +
                   d[4] * (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
        out[v] *= P;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Solver state                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nv[3];
    double vlo[3], vhi[3];
    int scheme;      /* 0: first-order upwind, 1: MUSCL with minmod limiter */
    int collision;   /* 0: exponential BGK, 1: explicit-Euler BGK, 2: off */
    int tau_mode;    /* 0: tau constant, 1: hard sphere tau = Kn T^(-1/2) / rho */
    double tau_or_kn;
    double inflow[5]; /* rho, ux, uy, uz, T of the inflow Maxwellian */
    double t_wall;    /* temperature of the diffuse wall (wall at rest) */
    int64_t korobov_p; /* collision 3: lattice points per velocity node (prime) */
    int64_t korobov_a; /* collision 3: lattice generator (0: the optimal one) */
    int lbm_q;         /* collision 4: 19 (D3Q19) or 27 (D3Q27) */
} or_params;

/* Korobov tables of one velocity grid: per node i and trial k, the partner
 * node j and the nodes l, m of the two post-collision velocities (-1 when a
 * velocity leaves the grid), and the weight W = V_box |g| / p; [i][k]. */
typedef struct {
    int64_t p, a, nv;
    int32_t *j, *l, *m;
    double *W;
} or_korobov;

typedef struct {
    const or_mesh *m;
    or_params p;
    or_vgrid g;
    double *f, *fn;      /* [n_rows][nv] */
    double *ghost_in;    /* corrected inflow Maxwellian */
    double *wall_m1;     /* corrected M(1, 0, T_wall) */
    double *sigma;       /* MUSCL slopes [n_rows][3][nv] */
    int flag;            /* sticky OR_ERR_NONPHYSICAL */
    /* Held cells.  A full solver holds every cell (row == cell, the arrays
     * below NULL).  A subset solver holds only the listed cells: f is known
     * exactly only where every value it depends on was held, and since
     * eq. (2) couples a cell to its face neighbours only, the exact region
     * shrinks by one face layer per step (two with MUSCL, whose slopes read
     * the neighbours' neighbours).  valid[] marks the rows still exact. */
    int64_t n_rows;
    int64_t *cells;      /* row -> cell */
    int64_t *row;        /* cell -> row, -1 when not held */
    uint8_t *valid, *valid_n, *sig_ok;
    or_korobov *kt;      /* collision 3 */
} or_solver;

/* ------------------------------------------------------------------------ */
/* Boltzmann collision integral on Korobov nodes (section 3.2, eqs. 3-6)     */
/* ------------------------------------------------------------------------ */
/*
 * The paper gives the structure of the discrete collision integral (eqs. 3-5:
 * per velocity node i a fixed list of M(i) trials, each with a partner node
 * gamma and a pair of nodes l, m, and weights b, c shared by all cells), not
 * the tables.  Reading used here (hard spheres of unit total cross section,
 * non-dimensional units of eq. 1):
 *   I(f)(xi) = int dxi* int dOmega/(4 pi) |g| (f(xi') f(xi*') - f(xi) f(xi*)),
 *   g = xi* - xi,  xi' = c + (|g|/2) n,  xi*' = c - (|g|/2) n,  c = (xi + xi*)/2,
 *   df/dt = I(f) / Kn.
 * For node i the 5-dimensional integral over the partner velocity (the
 * velocity box) and the direction n is a p-point Korobov lattice rule
 * (rank 1, generator a, p prime):
 *   z_d(k) = k a^d mod p,  d = 0..4, k = 0..p-1,
 *   shifted per node:  q_d = (z_d(k) + s_d(i)) mod p,  s_d(i) = (i + 1) c_d mod p,
 *                      c_d = (2654435761 mod p) (d + 1) mod p,
 *   x_d = (q_d + 1/2) / p,
 *   partner node j_b = floor(x_b N_b) = ((2 q_b + 1) N_b) div (2 p), b = 0, 1, 2,
 *   direction cos(theta) = 1 - 2 x_3, phi = 2 pi x_4,
 * the post-collision velocities belong to the nodes whose velocity cells hold
 * them (l, m; a trial whose xi' or xi*' leaves the grid contributes no gain),
 * and every trial weighs W = V_box |g| / p (the box volume over p, times the
 * relative speed; the sphere average cancels the 1/(4 pi)):
 *   B_i = sum_k W f_j          (eq. 4, the collision frequency)
 *   C_i = sum_k W f_l f_m      (eq. 5, the inverse-collision integral)
 *   I_i = -f_i P_i B_i + C_i   (eq. 6),  P_i = 1 + d0 + dx xi_x + dy xi_y + dz xi_z + d2 |xi|^2,
 * the five d from sum_i w psi_a I_i = 0, psi = (1, xi, |xi|^2) (conservation of
 * mass, momentum and energy), by Gauss elimination.  Time step (after the
 * transport): f' = f* + (dt / Kn) I(f*).
 * The generator is Korobov's optimal coefficient for the P_2 criterion:
 *   P_2(a) = -1 + (1/p) sum_k prod_d (1 + 2 pi^2 B_2(z_d(k) / p)),  B_2(x) = x^2 - x + 1/6,
 * the first a in 2, 3, ..., p - 1 with the smallest value (values within 1e-9
 * relative of each other count as equal).
 */
static int is_prime64(int64_t p) {
    if (p < 2) return 0;
    for (int64_t q = 2; q * q <= p; ++q)
        if (p % q == 0) return 0;
    return 1;
}

static double korobov_p2(int64_t p, int64_t a) {
    double sum = 0.0;
    for (int64_t k = 0; k < p; ++k) {
        double prod = 1.0;
        int64_t z = k;
        for (int d = 0; d < 5; ++d) {
            double x = (double)z / (double)p;
            prod *= 1.0 + 2.0 * M_PI * M_PI * (x * x - x + 1.0 / 6.0);
            z = (z * a) % p;
        }
        sum += prod;
    }
    return -1.0 + sum / (double)p;
}

/* Korobov's optimal generator for a p-point lattice in 5 dimensions, or -1 */
int64_t or_korobov_generator(int64_t p) {
    if (!is_prime64(p) || p < 5 || p >= (1ll << 31)) return -1;
    int64_t best = -1;
    double best_v = 0.0;
    for (int64_t a = 2; a < p; ++a) {
        double v = korobov_p2(p, a);
        /* a, -a, 1/a and -1/a (mod p) give the same lattice up to the order and
         * sign of the coordinates, hence the same value: values within 1e-9
         * relative are ties, and the first a wins */
        if (best < 0 || v < best_v - 1e-9 * fabs(best_v)) { best = a; best_v = v; }
    }
    return best;
}

/* node index of velocity component v along axis b, -1 outside the grid */
static int node_of(const or_vgrid *g, int b, double v) {
    double t = floor((v - g->lo[b]) / g->d[b]);
    if (t < 0.0 || t >= (double)g->n[b]) return -1;
    return (int)t;
}

static void korobov_free(or_korobov *t) {
    if (!t) return;
    free(t->j); free(t->l); free(t->m); free(t->W); free(t);
}

static or_korobov *korobov_build(const or_vgrid *g, int64_t p, int64_t a) {
    if (!is_prime64(p) || p < 5 || p >= (1ll << 31) || a < 1 || a >= p) return NULL;
    or_korobov *t = (or_korobov *)calloc(1, sizeof(or_korobov));
    int64_t nv = g->nv;
    t->p = p; t->a = a; t->nv = nv;
    t->j = (int32_t *)malloc((size_t)(nv * p) * sizeof(int32_t));
    t->l = (int32_t *)malloc((size_t)(nv * p) * sizeof(int32_t));
    t->m = (int32_t *)malloc((size_t)(nv * p) * sizeof(int32_t));
    t->W = (double *)malloc((size_t)(nv * p) * sizeof(double));
    double vbox = (g->hi[0] - g->lo[0]) * (g->hi[1] - g->lo[1]) * (g->hi[2] - g->lo[2]);
    int64_t apow[5], c[5];
    apow[0] = 1;
    for (int d = 1; d < 5; ++d) apow[d] = (apow[d - 1] * a) % p;
    for (int d = 0; d < 5; ++d) c[d] = ((2654435761ll % p) * (d + 1)) % p;
    for (int64_t i = 0; i < nv; ++i) {
        double xi[3];
        vgrid_xi(g, i, xi);
        int64_t sft[5];
        for (int d = 0; d < 5; ++d) sft[d] = ((i + 1) % p) * c[d] % p;
        for (int64_t k = 0; k < p; ++k) {
            int64_t q[5];
            for (int d = 0; d < 5; ++d) q[d] = ((k * apow[d]) % p + sft[d]) % p;
            int jb[3];
            for (int b = 0; b < 3; ++b) jb[b] = (int)(((2 * q[b] + 1) * g->n[b]) / (2 * p));
            int64_t j = ((int64_t)jb[0] * g->n[1] + jb[1]) * g->n[2] + jb[2];
            double xs[3] = {g->xi[0][jb[0]], g->xi[1][jb[1]], g->xi[2][jb[2]]};
            double gx = xs[0] - xi[0], gy = xs[1] - xi[1], gz = xs[2] - xi[2];
            double gg = sqrt(gx * gx + gy * gy + gz * gz);
            double x3 = ((double)q[3] + 0.5) / (double)p, x4 = ((double)q[4] + 0.5) / (double)p;
            double ct = 1.0 - 2.0 * x3;
            double st = sqrt(fmax(0.0, 1.0 - ct * ct));
            double ph = 2.0 * M_PI * x4;
            double n[3] = {st * cos(ph), st * sin(ph), ct};
            int l1[3], l2[3], ok = 1;
            for (int b = 0; b < 3; ++b) {
                double cb = 0.5 * (xi[b] + xs[b]);
                l1[b] = node_of(g, b, cb + 0.5 * gg * n[b]);
                l2[b] = node_of(g, b, cb - 0.5 * gg * n[b]);
                if (l1[b] < 0 || l2[b] < 0) ok = 0;
            }
            int64_t e = i * p + k;
            t->j[e] = (int32_t)j;
            t->l[e] = ok ? (int32_t)(((int64_t)l1[0] * g->n[1] + l1[1]) * g->n[2] + l1[2]) : -1;
            t->m[e] = ok ? (int32_t)(((int64_t)l2[0] * g->n[1] + l2[1]) * g->n[2] + l2[2]) : -1;
            t->W[e] = vbox * gg / (double)p;
        }
    }
    return t;
}

/* B (eq. 4) and C (eq. 5) of one cell's distribution */
static void korobov_terms(const or_korobov *t, const double *f, double *B, double *C) {
    for (int64_t i = 0; i < t->nv; ++i) {
        double b = 0.0, c = 0.0;
        for (int64_t k = 0; k < t->p; ++k) {
            int64_t e = i * t->p + k;
            b += t->W[e] * f[t->j[e]];
            if (t->l[e] >= 0) c += t->W[e] * f[t->l[e]] * f[t->m[e]];
        }
        B[i] = b;
        C[i] = c;
    }
}

/* I of eq. (6): the conservatively corrected collision integral of one cell */
static int korobov_integral(const or_vgrid *g, const or_korobov *t, const double *f, double *I, double *B, double *C) {
    korobov_terms(t, f, B, C);
    double G[25], r[5], d[5];
    memset(G, 0, sizeof G);
    memset(r, 0, sizeof r);
    for (int64_t i = 0; i < g->nv; ++i) {
        double xi[3];
        vgrid_xi(g, i, xi);
        double psi[5] = {1.0, xi[0], xi[1], xi[2], xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]};
        double fb = f[i] * B[i];
        for (int a = 0; a < 5; ++a) {
            r[a] += g->w * psi[a] * (C[i] - fb);
            for (int b = 0; b < 5; ++b) G[a * 5 + b] += g->w * psi[a] * psi[b] * fb;
        }
    }
    int rc = gauss_solve(5, G, r, d);
    if (rc) return rc;
    for (int64_t i = 0; i < g->nv; ++i) {
        double xi[3];
        vgrid_xi(g, i, xi);
        double P = 1.0 + d[0] + d[1] * xi[0] + d[2] * xi[1] + d[3] * xi[2] +
                   d[4] * (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
        I[i] = -f[i] * P * B[i] + C[i];
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Lattice Boltzmann subset (section 4)                                      */
/* ------------------------------------------------------------------------ */
/*
 * The LBM module is a DVM solver on a minimal velocity set (section 4): here
 * the 3x3x3 velocity grid on [-3/2, 3/2]^3, whose nodes are the lattice
 * vectors c in {-1, 0, 1}^3 with unit node volume, so the DVM moments are the
 * lattice sums rho = sum f, rho u = sum c f.  D3Q27 keeps all 27 nodes, D3Q19
 * drops the 8 corners (their f is zero and stays zero).  Weights by |c|^2 =
 * 0, 1, 2, 3: D3Q27 8/27, 2/27, 1/54, 1/216; D3Q19 1/3, 1/18, 1/36, 0.
 * Equilibrium of section 4 (second-order expansion, cs^2 = 1/3):
 *   f_eq = w rho (1 + c.u / cs^2 + (c.u)^2 / (2 cs^4) - |u|^2 / (2 cs^2)),
 * BGK collision (collision 4): f' = f_eq + (f* - f_eq) exp(-dt / tau), rho and
 * u from f*, tau = tau_or_kn.  Transport: the finite-volume upwind step of
 * eq. (2) on the octree, unchanged.
 */
static double lbm_weight(int q, const double c[3]) {
    int c2 = (int)(c[0] * c[0] + c[1] * c[1] + c[2] * c[2] + 0.5);
    if (q == 27) {
        static const double w27[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
        return w27[c2];
    }
    static const double w19[4] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0, 0.0};
    return w19[c2];
}

static int lbm_grid_ok(const or_params *p) {
    if (p->lbm_q != 19 && p->lbm_q != 27) return 0;
    for (int a = 0; a < 3; ++a)
        if (p->nv[a] != 3 || p->vlo[a] != -1.5 || p->vhi[a] != 1.5) return 0;
    return 1;
}

static void lbm_equilibrium(const or_vgrid *g, int q, double rho, const double u[3], double *out) {
    const double cs2 = 1.0 / 3.0;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int64_t v = 0; v < g->nv; ++v) {
        double c[3];
        vgrid_xi(g, v, c);
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        out[v] = lbm_weight(q, c) * rho * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
}

/* one LBM-BGK collision of a cell: rho, u of fs, exponential relaxation */
static int lbm_collide(const or_vgrid *g, const or_params *p, double dt, const double *fs, double *out, double *work) {
    double rho = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int64_t v = 0; v < g->nv; ++v) {
        double c[3];
        vgrid_xi(g, v, c);
        rho += fs[v];
        for (int a = 0; a < 3; ++a) m[a] += c[a] * fs[v];
    }
    if (!(rho > 0.0)) { memcpy(out, fs, (size_t)g->nv * sizeof(double)); return OR_ERR_NONPHYSICAL; }
    double u[3] = {m[0] / rho, m[1] / rho, m[2] / rho};
    lbm_equilibrium(g, p->lbm_q, rho, u, work);
    double e = exp(-dt / p->tau_or_kn);
    for (int64_t v = 0; v < g->nv; ++v) out[v] = work[v] + (fs[v] - work[v]) * e;
    return OR_OK;
}

static int64_t row_of(const or_solver *s, int64_t c) { return s->row ? s->row[c] : c; }
static int64_t cell_of(const or_solver *s, int64_t r) { return s->cells ? s->cells[r] : r; }
static const double *f_of(const or_solver *s, int64_t c) { return s->f + row_of(s, c) * s->g.nv; }

static int target_of_prim(const double prim[5], double target[5]) {
    double rho = prim[0], T = prim[4];
    if (!(rho > 0.0) || !(T > 0.0)) return OR_ERR_NONPHYSICAL;
    target[0] = rho;
    for (int a = 0; a < 3; ++a) target[1 + a] = rho * prim[1 + a];
    target[4] = 0.5 * rho * (prim[1] * prim[1] + prim[2] * prim[2] + prim[3] * prim[3]) + 1.5 * rho * T;
    return OR_OK;
}

void or_solver_free(or_solver *s) {
    if (!s) return;
    free(s->f); free(s->fn); free(s->ghost_in); free(s->wall_m1); free(s->sigma);
    free(s->cells); free(s->row); free(s->valid); free(s->valid_n); free(s->sig_ok);
    korobov_free(s->kt);
    vgrid_free(&s->g);
    free(s);
}

/* n_sub < 0: every cell; else the n_sub cells listed in ascending order */
int or_solver_new_subset(const or_mesh *m, const or_params *p, int64_t n_sub, const int64_t *sub, or_solver **out) {
    for (int a = 0; a < 3; ++a)
        if (p->nv[a] < 1 || !(p->vhi[a] > p->vlo[a])) return OR_ERR_ARG;
    if (n_sub >= 0) {
        if (n_sub < 1 || !sub) return OR_ERR_ARG;
        for (int64_t r = 0; r < n_sub; ++r)
            if (sub[r] < 0 || sub[r] >= m->n_cells || (r && sub[r] <= sub[r - 1])) return OR_ERR_ARG;
    }
    or_solver *s = (or_solver *)calloc(1, sizeof(or_solver));
    s->m = m;
    s->p = *p;
    vgrid_init(&s->g, p->nv, p->vlo, p->vhi);
    s->n_rows = n_sub < 0 ? m->n_cells : n_sub;
    if (n_sub >= 0) {
        s->cells = (int64_t *)malloc((size_t)n_sub * sizeof(int64_t));
        memcpy(s->cells, sub, (size_t)n_sub * sizeof(int64_t));
        s->row = (int64_t *)malloc((size_t)m->n_cells * sizeof(int64_t));
        for (int64_t c = 0; c < m->n_cells; ++c) s->row[c] = -1;
        for (int64_t r = 0; r < n_sub; ++r) s->row[sub[r]] = r;
        s->valid = (uint8_t *)malloc((size_t)n_sub);
        s->valid_n = (uint8_t *)malloc((size_t)n_sub);
        s->sig_ok = (uint8_t *)malloc((size_t)n_sub);
        memset(s->valid, 1, (size_t)n_sub);
        memset(s->sig_ok, 1, (size_t)n_sub);
    }
    size_t sz = (size_t)s->n_rows * (size_t)s->g.nv;
    s->f = (double *)calloc(sz, sizeof(double));
    s->fn = (double *)calloc(sz, sizeof(double));
    s->ghost_in = (double *)calloc((size_t)s->g.nv, sizeof(double));
    s->wall_m1 = (double *)calloc((size_t)s->g.nv, sizeof(double));
    if (p->scheme == 1) s->sigma = (double *)calloc(sz * 3, sizeof(double));
    /* ghost distributions, built only when the mesh has such faces (a
     * degenerate velocity grid cannot carry a corrected Maxwellian) */
    int has_in = 0, has_wall = 0;
    for (int64_t t = 0; t < m->n_cells * 6; ++t) {
        has_in |= m->type[t] == OR_FACE_INFLOW;
        has_wall |= m->type[t] == OR_FACE_WALL;
    }
    double tgt[5];
    int rc = OR_OK;
    if (has_in) {
        rc = target_of_prim(p->inflow, tgt);
        if (!rc) rc = corrected_maxwellian(&s->g, tgt, s->ghost_in);
    }
    double pw[5] = {1.0, 0.0, 0.0, 0.0, p->t_wall};
    if (!rc && has_wall) {
        rc = target_of_prim(pw, tgt);
        if (!rc) rc = corrected_maxwellian(&s->g, tgt, s->wall_m1);
    }
    if (!rc && p->collision == 4 && !lbm_grid_ok(p)) rc = OR_ERR_ARG;
    if (!rc && p->collision == 3) {
        int64_t a = p->korobov_a ? p->korobov_a : or_korobov_generator(p->korobov_p);
        s->kt = korobov_build(&s->g, p->korobov_p, a);
        if (!s->kt || !(p->tau_or_kn > 0.0)) rc = OR_ERR_ARG;
    }
    if (rc) { or_solver_free(s); return rc; }
    *out = s;
    return OR_OK;
}

int or_solver_new(const or_mesh *m, const or_params *p, or_solver **out) {
    return or_solver_new_subset(m, p, -1, NULL, out);
}

int64_t or_solver_nv(const or_solver *s) { return s->g.nv; }
int64_t or_solver_rows(const or_solver *s) { return s->n_rows; }
void or_set_f(or_solver *s, const double *f) { memcpy(s->f, f, (size_t)s->n_rows * s->g.nv * sizeof(double)); }
void or_get_f(const or_solver *s, double *f) { memcpy(f, s->f, (size_t)s->n_rows * s->g.nv * sizeof(double)); }
int or_flag(const or_solver *s) { return s->flag; }
/* 1 per row whose state is exact (always 1 for a full solver) */
void or_valid(const or_solver *s, uint8_t *out) {
    if (s->valid) memcpy(out, s->valid, (size_t)s->n_rows);
    else memset(out, 1, (size_t)s->n_rows);
}

/* LBM: f := f_eq(rho, u) per held cell; prim is [4][n_rows] (rho, ux, uy, uz) */
int or_init_lbm(or_solver *s, const double *prim) {
    if (s->p.collision != 4) return OR_ERR_ARG;
    int64_t n = s->n_rows;
    for (int64_t c = 0; c < n; ++c) {
        double u[3] = {prim[1 * n + c], prim[2 * n + c], prim[3 * n + c]};
        if (!(prim[c] > 0.0)) return OR_ERR_NONPHYSICAL;
        lbm_equilibrium(&s->g, s->p.lbm_q, prim[c], u, s->f + c * s->g.nv);
    }
    return OR_OK;
}

/* f := corrected Maxwellian of (rho, ux, uy, uz, T) per held cell; prim is [5][n_rows] */
int or_init_maxwellian(or_solver *s, const double *prim) {
    int64_t n = s->n_rows;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : err)
    for (int64_t c = 0; c < n; ++c) {
        double pc[5], tgt[5];
        for (int a = 0; a < 5; ++a) pc[a] = prim[a * n + c];
        int rc = target_of_prim(pc, tgt);
        if (!rc) rc = corrected_maxwellian(&s->g, tgt, s->f + c * s->g.nv);
        if (rc) err |= 1;
    }
    return err ? OR_ERR_NONPHYSICAL : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Transport: eq. (2) in flux form                                          */
/* ------------------------------------------------------------------------ */

/* sign of the outward normal of face f (-x,+x,-y,+y,-z,+z) */
static double face_sign(int f) { return (f % 2) ? 1.0 : -1.0; }

/*
 * Diffuse-wall density for cell c and wall face f (wall at rest, temperature
 * T_wall): re-emitted molecules carry rho_w times the corrected unit-density
 * wall Maxwellian, with rho_w chosen so that no mass crosses the wall:
 *   rho_w = sum_{xi.n>0} (xi.n) f_face_i / sum_{xi.n<0} |xi.n| M1_i,
 * n the outward normal of the cell, f_face the value leaving the cell.
 */
static double wall_density(const or_solver *s, int64_t c, int f) {
    const or_vgrid *g = &s->g;
    double num = 0.0, den = 0.0, sg = face_sign(f);
    int axis = f / 2;
    const double *fc = f_of(s, c);
    for (int64_t v = 0; v < g->nv; ++v) {
        double xi[3];
        vgrid_xi(g, v, xi);
        double xn = sg * xi[axis];
        if (xn > 0.0) num += xn * fc[v]; /* MUSCL slopes vanish next to a wall */
        else if (xn < 0.0) den += -xn * s->wall_m1[v];
    }
    return num / den;
}

/*
 * MUSCL slope of cell c along `axis` for velocity v (the paper is silent on
 * the reconstruction; reading: minmod of the one-sided differences to the
 * face-neighbour values, a FINER face taking the mean of its 4 leaves, with
 * centre distances h (SAME or boundary), 3h/4 (FINER), 3h/2 (COARSER); zero in
 * leaves that touch a wall; ghost cells carry no slope).
 */
static double minmod(double a, double b) {
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}
static double neighbour_mean(const or_solver *s, int64_t c, int f, int64_t v, double *dist) {
    const or_mesh *m = s->m;
    double h = cell_h(m, c);
    int ty = m->type[c * 6 + f];
    const int32_t *nb = &m->nbr[(c * 6 + f) * 4];
    switch (ty) {
    case OR_FACE_SAME: *dist = h; return f_of(s, nb[0])[v];
    case OR_FACE_COARSER: *dist = 1.5 * h; return f_of(s, nb[0])[v];
    case OR_FACE_FINER:
        *dist = 0.75 * h;
        return 0.25 * (f_of(s, nb[0])[v] + f_of(s, nb[1])[v] + f_of(s, nb[2])[v] + f_of(s, nb[3])[v]);
    case OR_FACE_INFLOW: *dist = h; return s->ghost_in[v];
    default: *dist = h; return f_of(s, c)[v]; /* OUTFLOW: zero gradient */
    }
}

/* subset solver: 1 when every face neighbour of cell c is held and has
 * flag ok[] set (domain faces need nothing) */
static int neighbours_ok(const or_solver *s, int64_t c, const uint8_t *ok) {
    const or_mesh *m = s->m;
    for (int f = 0; f < 6; ++f) {
        int ty = m->type[c * 6 + f];
        int k = ty == OR_FACE_FINER ? 4 : (ty == OR_FACE_SAME || ty == OR_FACE_COARSER) ? 1 : 0;
        for (int q = 0; q < k; ++q) {
            int64_t r = s->row[m->nbr[(c * 6 + f) * 4 + q]];
            if (r < 0 || !ok[r]) return 0;
        }
    }
    return 1;
}

static void or_muscl_sigma(or_solver *s) {
    const or_mesh *m = s->m;
    int64_t nv = s->g.nv, n = s->n_rows;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n; ++r) {
        int64_t c = cell_of(s, r);
        if (s->valid) {
            s->sig_ok[r] = s->valid[r] && neighbours_ok(s, c, s->valid);
            if (!s->sig_ok[r]) continue;
        }
        int wall = 0;
        for (int f = 0; f < 6; ++f) wall |= m->type[c * 6 + f] == OR_FACE_WALL;
        for (int axis = 0; axis < 3; ++axis)
            for (int64_t v = 0; v < nv; ++v) {
                double sig = 0.0;
                if (!wall) {
                    double dm, dp;
                    double fm = neighbour_mean(s, c, 2 * axis, v, &dm);
                    double fp = neighbour_mean(s, c, 2 * axis + 1, v, &dp);
                    double fc = f_of(s, c)[v];
                    sig = minmod((fc - fm) / dm, (fp - fc) / dp);
                }
                s->sigma[(r * 3 + axis) * nv + v] = sig;
            }
    }
}

/* value of cell c's distribution at its face f for velocity v */
static double face_value(const or_solver *s, int64_t c, int f, int64_t v) {
    double val = f_of(s, c)[v];
    if (s->p.scheme == 1) {
        double h = cell_h(s->m, c);
        val += face_sign(f) * 0.5 * h * s->sigma[(row_of(s, c) * 3 + f / 2) * s->g.nv + v];
    }
    return val;
}

/* opposite face: the neighbour's face that coincides with face f of the cell */
static int opposite(int f) { return f ^ 1; }

/*
 * One explicit-Euler transport step (eq. 2 in flux form):
 *   f*_{c,i} = f_{c,i} - dt/V_c * sum_faces sum_subfaces A (xi_i . n) f_up,
 * with f_up the cell's own face value when xi.n > 0 and the upwind neighbour's
 * (or the ghost's) when xi.n < 0.  A is h^2 for a SAME or COARSER face and
 * (h/2)^2 for each of the 4 sub-faces of a FINER face; V = h^3.
 */
static void transport(or_solver *s, double dt) {
    const or_mesh *m = s->m;
    const or_vgrid *g = &s->g;
    int64_t nv = g->nv, n = s->n_rows;
    if (s->p.scheme == 1) or_muscl_sigma(s);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n; ++r) {
        int64_t c = cell_of(s, r);
        if (s->valid) { /* subset: exact only if everything read below is exact */
            const uint8_t *ok = s->p.scheme == 1 ? s->sig_ok : s->valid;
            s->valid_n[r] = ok[r] && neighbours_ok(s, c, ok);
            if (!s->valid_n[r]) {
                memcpy(s->fn + r * nv, s->f + r * nv, (size_t)nv * sizeof(double));
                continue;
            }
        }
        double h = cell_h(m, c), V = h * h * h;
        double rho_w[6] = {0, 0, 0, 0, 0, 0};
        for (int f = 0; f < 6; ++f)
            if (m->type[c * 6 + f] == OR_FACE_WALL) rho_w[f] = wall_density(s, c, f);
        for (int64_t v = 0; v < nv; ++v) {
            double xi[3];
            vgrid_xi(g, v, xi);
            double acc = 0.0;
            for (int f = 0; f < 6; ++f) {
                double xn = face_sign(f) * xi[f / 2];
                if (xn == 0.0) continue;
                int ty = m->type[c * 6 + f];
                const int32_t *nb = &m->nbr[(c * 6 + f) * 4];
                if (xn > 0.0) { /* leaving the cell: own face value over the whole face */
                    if (ty == OR_FACE_FINER)
                        for (int q = 0; q < 4; ++q) acc += (0.5 * h) * (0.5 * h) * xn * face_value(s, c, f, v);
                    else
                        acc += h * h * xn * face_value(s, c, f, v);
                    continue;
                }
                switch (ty) { /* entering: upwind value */
                case OR_FACE_SAME:
                case OR_FACE_COARSER: acc += h * h * xn * face_value(s, nb[0], opposite(f), v); break;
                case OR_FACE_FINER:
                    for (int q = 0; q < 4; ++q) acc += (0.5 * h) * (0.5 * h) * xn * face_value(s, nb[q], opposite(f), v);
                    break;
                case OR_FACE_INFLOW: acc += h * h * xn * s->ghost_in[v]; break;
                case OR_FACE_OUTFLOW: acc += h * h * xn * s->f[r * nv + v]; break;
                case OR_FACE_WALL: acc += h * h * xn * rho_w[f] * s->wall_m1[v]; break;
                }
            }
            s->fn[r * nv + v] = s->f[r * nv + v] - dt / V * acc;
        }
    }
    if (s->valid) { uint8_t *t = s->valid; s->valid = s->valid_n; s->valid_n = t; }
}

/* ------------------------------------------------------------------------ */
/* Collision: BGK relaxation toward the corrected Maxwellian                */
/* ------------------------------------------------------------------------ */

static double relaxation_time(const or_params *p, double rho, double T) {
    if (p->tau_mode == 0) return p->tau_or_kn;
    return p->tau_or_kn * pow(T, -0.5) / rho; /* hard sphere: viscosity ~ T^(1/2) */
}

/*
 * One BGK step for one cell (section 4 form I = -(f - f_eq)/tau with f_eq the
 * conservatively corrected discrete Maxwellian of the cell's own moments):
 *   EXP:   f' = Mt + (f* - Mt) exp(-dt/tau)   (exact solution over dt)
 *   EULER: f' = f* + dt/tau (Mt - f*)
 *   OFF:   f' = f*
 */
static int collide_cell(const or_vgrid *g, const or_params *p, const or_korobov *kt, double dt, const double *fs,
                        double *out, double *work) {
    int64_t nv = g->nv;
    if (p->collision == 2) { memcpy(out, fs, (size_t)nv * sizeof(double)); return OR_OK; }
    if (p->collision == 4) return lbm_collide(g, p, dt, fs, out, work);
    double mom[5], rho, u[3], T;
    moments_of(g, fs, mom);
    int rc = primitive_of(mom, &rho, u, &T);
    if (rc) { memcpy(out, fs, (size_t)nv * sizeof(double)); return rc; }
    if (p->collision == 3) { /* Boltzmann integral on Korobov nodes, explicit Euler */
        double *I = work, *B = work + nv, *C = work + 2 * nv;
        rc = korobov_integral(g, kt, fs, I, B, C);
        if (rc) { memcpy(out, fs, (size_t)nv * sizeof(double)); return rc; }
        for (int64_t v = 0; v < nv; ++v) out[v] = fs[v] + dt / p->tau_or_kn * I[v];
        return OR_OK;
    }
    rc = corrected_maxwellian(g, mom, work);
    if (rc) { memcpy(out, fs, (size_t)nv * sizeof(double)); return rc; }
    double tau = relaxation_time(p, rho, T);
    if (p->collision == 0) {
        double e = exp(-dt / tau);
        for (int64_t v = 0; v < nv; ++v) out[v] = work[v] + (fs[v] - work[v]) * e;
    } else {
        for (int64_t v = 0; v < nv; ++v) out[v] = fs[v] + dt / tau * (work[v] - fs[v]);
    }
    return OR_OK;
}

/* one full step: transport, then collision (Lie splitting) */
int or_step(or_solver *s, double dt, int n_steps) {
    int64_t n = s->n_rows, nv = s->g.nv;
    for (int it = 0; it < n_steps; ++it) {
        transport(s, dt);
        int err = 0;
#pragma omp parallel reduction(| : err)
        {
            double *work = (double *)malloc((size_t)(3 * nv) * sizeof(double));
#pragma omp for schedule(dynamic, 16)
            for (int64_t r = 0; r < n; ++r) {
                if (s->valid && !s->valid[r]) { /* not exact any more: carried, not collided */
                    memcpy(s->f + r * nv, s->fn + r * nv, (size_t)nv * sizeof(double));
                    continue;
                }
                if (collide_cell(&s->g, &s->p, s->kt, dt, s->fn + r * nv, s->f + r * nv, work)) err |= 1;
            }
            free(work);
        }
        if (err) s->flag = OR_ERR_NONPHYSICAL;
    }
    return s->flag;
}

/* transport only, result left in the state (used to expose f* to tests) */
void or_transport(or_solver *s, double dt) {
    transport(s, dt);
    double *t = s->f; s->f = s->fn; s->fn = t;
}

/* moments [5][n_rows]: rho, rho ux, rho uy, rho uz, E of the current f */
void or_moments(const or_solver *s, double *out) {
    int64_t n = s->n_rows;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        double mom[5];
        moments_of(&s->g, s->f + r * s->g.nv, mom);
        for (int a = 0; a < 5; ++a) out[a * n + r] = mom[a];
    }
}

/* global conserved quantities sum_c V_c (rho, rho u, E) over the held cells, in cell order */
void or_global_sums(const or_solver *s, double out[5]) {
    int64_t n = s->n_rows;
    double *mom = (double *)malloc((size_t)5 * n * sizeof(double));
    or_moments(s, mom);
    for (int a = 0; a < 5; ++a) out[a] = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        double h = cell_h(s->m, cell_of(s, r)), V = h * h * h;
        for (int a = 0; a < 5; ++a) out[a] += V * mom[a * n + r];
    }
    free(mom);
}

/* largest stable step of unsplit 3D first-order upwind at Courant number cfl:
 * dt = cfl * h_min / max_i (|xi_x| + |xi_y| + |xi_z|) */
double or_dt_cfl(const or_solver *s, double cfl) {
    double hmin = 1e300, smax = 0.0;
    for (int64_t c = 0; c < s->m->n_cells; ++c) hmin = fmin(hmin, cell_h(s->m, c));
    for (int64_t v = 0; v < s->g.nv; ++v) {
        double xi[3];
        vgrid_xi(&s->g, v, xi);
        smax = fmax(smax, fabs(xi[0]) + fabs(xi[1]) + fabs(xi[2]));
    }
    return cfl * hmin / smax;
}

/* ---- single-cell entry points for the collision pins ---- */

int or_cell_maxwellian(const int nvx[3], const double lo[3], const double hi[3], const double prim[5], double *out) {
    or_vgrid g;
    vgrid_init(&g, nvx, lo, hi);
    double tgt[5];
    int rc = target_of_prim(prim, tgt);
    if (!rc) rc = corrected_maxwellian(&g, tgt, out);
    vgrid_free(&g);
    return rc;
}

int or_cell_moments(const int nvx[3], const double lo[3], const double hi[3], const double *f, double mom[5]) {
    or_vgrid g;
    vgrid_init(&g, nvx, lo, hi);
    moments_of(&g, f, mom);
    vgrid_free(&g);
    return OR_OK;
}

int or_cell_collide(const or_params *p, double dt, const double *fs, double *out) {
    or_vgrid g;
    vgrid_init(&g, p->nv, p->vlo, p->vhi);
    or_korobov *kt = NULL;
    if (p->collision == 3) {
        int64_t a = p->korobov_a ? p->korobov_a : or_korobov_generator(p->korobov_p);
        kt = korobov_build(&g, p->korobov_p, a);
        if (!kt) { vgrid_free(&g); return OR_ERR_ARG; }
    }
    double *work = (double *)malloc((size_t)(3 * g.nv) * sizeof(double));
    int rc = collide_cell(&g, p, kt, dt, fs, out, work);
    free(work);
    korobov_free(kt);
    vgrid_free(&g);
    return rc;
}

/* Korobov tables of a velocity grid ([nv][p] each; any output may be NULL) */
int or_korobov_tables(const int nvx[3], const double lo[3], const double hi[3], int64_t p, int64_t a, int32_t *j,
                      int32_t *l, int32_t *m, double *W) {
    or_vgrid g;
    vgrid_init(&g, nvx, lo, hi);
    or_korobov *t = korobov_build(&g, p, a);
    vgrid_free(&g);
    if (!t) return OR_ERR_ARG;
    size_t n = (size_t)(t->nv * p);
    if (j) memcpy(j, t->j, n * sizeof(int32_t));
    if (l) memcpy(l, t->l, n * sizeof(int32_t));
    if (m) memcpy(m, t->m, n * sizeof(int32_t));
    if (W) memcpy(W, t->W, n * sizeof(double));
    korobov_free(t);
    return OR_OK;
}

/* one cell: B (eq. 4), C (eq. 5) and the corrected integral I (eq. 6) */
int or_korobov_cell(const int nvx[3], const double lo[3], const double hi[3], int64_t p, int64_t a, const double *f,
                    double *I, double *B, double *C) {
    or_vgrid g;
    vgrid_init(&g, nvx, lo, hi);
    or_korobov *t = korobov_build(&g, p, a);
    int rc = OR_ERR_ARG;
    if (t) rc = korobov_integral(&g, t, f, I, B, C);
    korobov_free(t);
    vgrid_free(&g);
    return rc;
}

void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
