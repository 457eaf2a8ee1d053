/*
 * dvm.h -- C interface of the MI355X DVM-BGK octree library.
 *
 * The library advances the discrete-velocity (DVM) form of the kinetic
 * equation (eq. 1 of Zabelok, Arslanbekov & Kolobov, arXiv:1503.00707) on a
 * 2:1-balanced forest of octrees (section 2.1).  One step is
 *   1. upwind finite-volume transport of f(x, xi) across leaf faces for every
 *      discrete velocity (eq. 2, section 3.1), first order or minmod-MUSCL;
 *   2. a per-cell FP64 reduction to the conserved moments (rho, rho u, E)
 *      (the moment sums of the correction kernel, section 3.2);
 *   3. BGK relaxation (the BGK form of section 4) toward a discrete
 *      Maxwellian corrected by the polynomial P of eq. (6) so that mass,
 *      momentum and energy are conserved to rounding (section 3.2).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int status (DVM_OK or a negative DVM_ERR_*);
 *     no C++ exception crosses the interface.  dvm_last_error() returns a
 *     thread-local text for the last failure on the calling thread.
 *   - Argument errors are detected synchronously, before anything is
 *     enqueued.  Device-side conditions (a cell with rho <= 0, T <= 0 or NaN)
 *     set a device flag that the synchronising dvm_check() reports as
 *     DVM_ERR_NONPHYSICAL.
 *   - Device work is enqueued on the caller's hipStream_t (passed as void*;
 *     NULL is the default stream) and is asynchronous.
 *   - Ownership: the caller owns every device buffer (allocated e.g. by
 *     PyTorch) and keeps it alive while the solver uses it.  The library owns
 *     only host objects, released by dvm_destroy_*.
 *   - Geometry: leaf (level l, i, j, k) is the cube [i, i+1) x [j, j+1) x
 *     [k, k+1) scaled by h0 * 2^-l; root cubes form an nx x ny x nz lattice.
 *     Domain faces are ordered -x, +x, -y, +y, -z, +z.
 *   - Velocity grid: cell centres xi_k = lo + (k + 1/2)(hi - lo)/N per axis
 *     (section 3: f at cell centres of a uniform Cartesian velocity grid).
 *     The device path requires the same even N on all axes and lo = -hi per
 *     axis.  Internally f[cell][v] keeps the 8 velocity sign groups ("octants")
 *     contiguous, (-,-,-) first and the z sign fastest (section 3.1, step 1);
 *     inside an octant slot s = (ax*NH + ay)*NH + az, NH = N/2, addresses the
 *     node with |xi_b| = (a_b + 1/2) d_b.  dvm_f_to_canonical() converts to
 *     the canonical order i = (kx*N + ky)*N + kz.
 */
#ifndef DVM_H
#define DVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define DVM_OK 0
#define DVM_ERR_ARG (-1)            /* invalid argument */
#define DVM_ERR_UNBALANCED (-2)     /* leaves violate the 2:1 rule */
#define DVM_ERR_NOT_PARTITION (-3)  /* leaves overlap, leave a gap or leave the domain */
#define DVM_ERR_WORKSPACE (-4)      /* a bound buffer is missing or too small */
#define DVM_ERR_NONPHYSICAL (-5)    /* rho <= 0, T <= 0 or NaN met on the device */
#define DVM_ERR_DEVICE (-6)         /* a HIP runtime call failed */
#define DVM_ERR_UNSUPPORTED (-7)    /* valid but not provided by the device path */

/* ---- domain boundary kinds (per domain face) ---- */
#define DVM_BC_PERIODIC 0  /* both faces of an axis must be periodic */
#define DVM_BC_INFLOW 1    /* ghost = corrected Maxwellian of the inflow state */
#define DVM_BC_OUTFLOW 2   /* ghost = the cell's own f (zero gradient) */
#define DVM_BC_WALL 3      /* diffuse wall at rest, temperature t_wall */

/* ---- face kinds in the exported tables ---- */
#define DVM_FACE_SAME 0     /* one neighbour of the same level */
#define DVM_FACE_COARSER 1  /* one neighbour one level coarser */
#define DVM_FACE_FINER 2    /* four neighbours one level finer, ascending Morton key */
#define DVM_FACE_INFLOW 3
#define DVM_FACE_OUTFLOW 4
#define DVM_FACE_WALL 5     /* domain wall or a fluid-solid face */

/* ---- solver options ---- */
#define DVM_PREC_FP64 0         /* f stored and transported in FP64 */
#define DVM_PREC_FP32 1         /* f in FP32; moments, Maxwellian, correction in FP64 */
#define DVM_SCHEME_UPWIND1 0
#define DVM_SCHEME_MUSCL 1      /* minmod-limited linear reconstruction, formed inside the
                                   step from two face hops per axis (no extra buffers) */
#define DVM_COLL_EXP 0          /* f' = Mt + (f* - Mt) exp(-dt/tau) */
#define DVM_COLL_EULER 1        /* f' = f* + dt/tau (Mt - f*) */
#define DVM_COLL_OFF 2          /* f' = f* */
#define DVM_COLL_KOROBOV 3      /* f' = f* + dt/Kn I(f*), I the hard-sphere Boltzmann integral on
                                   Korobov lattice nodes with the correction of eq. (6)
                                   (section 3.2); Kn = tau_or_kn; N = 4, 8 or 12 */
#define DVM_FLUX_GRID 0         /* hybrid fluid-fluid faces: half-range sums of Mt(U) over the
                                   discrete velocity set (exactly what a kinetic neighbour sees) */
#define DVM_FLUX_CLOSED 1       /* hybrid fluid-fluid faces: the continuous half-range integrals
                                   of the Maxwellian of U (erf / exp closed form, kinetic
                                   flux-vector splitting); kinetic-fluid faces keep the sums */
#define DVM_TAU_CONST 0         /* tau = tau_or_kn */
#define DVM_TAU_HS 1            /* tau = Kn T^(-1/2) / rho (hard sphere) */

typedef struct dvm_mesh dvm_mesh;
typedef struct dvm_solver dvm_solver;
typedef struct dvm_batch dvm_batch;
typedef struct dvm_mlp dvm_mlp;

typedef struct {
    int32_t base[3];          /* root cubes per axis, each >= 1 */
    double h0;                /* root cube edge, > 0 */
    int32_t bc[6];            /* DVM_BC_* per domain face */
    int64_t n_leaves;
    const uint8_t *level;     /* [n_leaves], host */
    const int32_t *ijk;       /* [n_leaves][3], host, coordinates at the leaf's level */
    const uint8_t *solid;     /* [n_leaves] or NULL; nonzero = inside a body */
} dvm_mesh_desc;

typedef struct {
    int64_t n_leaves;         /* all leaves */
    int64_t n_cells;          /* fluid leaves (the cells that carry f) */
    int32_t max_level;
    double h_min;
    int64_t n_faces[6];       /* count of faces of each DVM_FACE_* kind */
} dvm_mesh_info_t;

typedef struct {
    int32_t nv;               /* velocity nodes per axis (even) */
    double vmax[3];           /* grid on [-vmax, vmax] per axis */
    int32_t precision;        /* DVM_PREC_* */
    int32_t scheme;           /* DVM_SCHEME_* */
    int32_t collision;        /* DVM_COLL_* */
    int32_t tau_mode;         /* DVM_TAU_* */
    double tau_or_kn;
    double inflow[5];         /* rho, ux, uy, uz, T of the inflow state */
    double t_wall;            /* diffuse-wall temperature */
    int32_t check_every;      /* global sums every k steps (0: never) */
    int32_t hybrid;           /* 1: workspace for dvm_hybrid_step (masks, flux sums) */
    int32_t korobov_p;        /* DVM_COLL_KOROBOV: lattice points per velocity node (a prime) */
    int32_t korobov_a;        /* DVM_COLL_KOROBOV: lattice generator; 0: Korobov's optimal one */
    int32_t fluid_flux;       /* DVM_FLUX_*: fluxes between two fluid cells of dvm_hybrid_step */
} dvm_params;

typedef struct {
    size_t f_bytes;           /* one state buffer; two are bound (ping-pong) */
    size_t moments_bytes;     /* FP64 [5][n_cells] */
    size_t tables_bytes;      /* device mesh tables */
    size_t ws_bytes;          /* ghost tables, flags, reduction partials, selection list,
                                 hybrid masks and flux records, Korobov trial table */
    int64_t n_cells;
    int64_t nv_total;         /* N^3 */
} dvm_sizes;

typedef struct {
    double sums[5];           /* sum_c V_c (rho, rho ux, rho uy, rho uz, E), FP64 */
    int32_t nonphysical;      /* 1 if the device flag was raised */
    int64_t steps;            /* steps taken since dvm_bind */
} dvm_diag;

/*
 * Boltzmann collision integral on Korobov lattice nodes (DVM_COLL_KOROBOV,
 * section 3.2, eqs. 3-6).  The tables of eqs. 3-5 (per velocity node i and
 * trial k: the partner node j and the post-collision nodes l, m) are built
 * on the host when the solver is created and live in its workspace.  For
 * node i and trial k of a p-point rank-1 lattice in 5 dimensions (generator
 * a): q_d = (k a^d + (i + 1) c_d) mod p, c_d = (2654435761 mod p)(d + 1) mod p;
 * j_b = floor((q_b + 1/2) N / p) (b = 0..2); n from cos(theta) = 1 - 2 (q_3 +
 * 1/2)/p, phi = 2 pi (q_4 + 1/2)/p; l, m the nodes whose velocity cells hold
 * (xi_i + xi_j)/2 +- |xi_j - xi_i|/2 n (-1: no gain term); weight
 * V_box |xi_j - xi_i| / p.  Canonical velocity indices; node velocities
 * -vmax + (k + 1/2) 2 vmax / N.
 * dvm_korobov_generator -- Korobov's optimal generator of a p-point lattice
 * in 5 dimensions (smallest P_2 merit, first of ties); DVM_ERR_ARG unless p is
 * a prime in [5, 2^31).
 * dvm_korobov_tables -- the tables [N^3][p] of the velocity grid N^3 on
 * [-vmax, vmax]^3 (host arrays), for tests and inspection.
 */
int dvm_korobov_generator(int64_t p, int64_t *a);
int dvm_korobov_tables(int32_t nv, double vmax, int64_t p, int64_t a, int32_t *j, int32_t *l, int32_t *m);

/* Text of the last error on this thread ("" if none). */
const char *dvm_last_error(void);

/*
 * dvm_balance -- refine a partition until the 2:1 rule holds between leaves
 * that share a face, an edge or a corner (section 2.1: levels of direct and
 * diagonal neighbours differ by at most one).  Periodic axes (bc) wrap.
 * Writes at most `cap` leaves (level_out[cap], ijk_out[cap][3], host) in
 * Morton order; *n_out is always set.  Returns DVM_ERR_WORKSPACE if cap is
 * too small, DVM_ERR_NOT_PARTITION if the input is not a partition.
 */
int dvm_balance(const dvm_mesh_desc *d, int64_t cap, int64_t *n_out, uint8_t *level_out, int32_t *ijk_out);

/*
 * dvm_create_mesh -- validate a leaf list (exact partition, 2:1 balanced) and
 * build the Morton ("N-order", section 2.1) cell order and the per-cell face
 * tables used by the transport (the stencil of eq. 2, section 3.1 step 4).
 * Host only; copies what it needs from *d.
 */
int dvm_create_mesh(const dvm_mesh_desc *d, dvm_mesh **out);
int dvm_mesh_info(const dvm_mesh *m, dvm_mesh_info_t *out);

/*
 * dvm_mesh_export -- host copies of the tables, for tests.  Any pointer may be
 * NULL.  Per fluid cell c (Morton rank): input[c] = index in the caller's
 * leaf list, key[c] = Morton key on the finest lattice (x bit lowest),
 * type[c][6] = DVM_FACE_*, nbr[c][6][4] = neighbour cells (-1 padding).
 */
int dvm_mesh_export(const dvm_mesh *m, int64_t *input, uint64_t *key, uint8_t *type, int32_t *nbr);
void dvm_destroy_mesh(dvm_mesh *m);

/*
 * dvm_create_solver -- a solver for one mesh (which must outlive it).
 * DVM_ERR_UNSUPPORTED for a velocity grid the device path does not provide.
 */
int dvm_create_solver(const dvm_mesh *m, const dvm_params *p, dvm_solver **out);
int dvm_buffer_sizes(const dvm_solver *s, dvm_sizes *out);

/*
 * dvm_bind -- device buffers owned by the caller: two state buffers of
 * f_bytes (f_a holds the current state after binding), the FP64 moments
 * [5][n_cells], the mesh tables and the workspace, sizes from
 * dvm_buffer_sizes.  Pointers must be 256-byte aligned.
 */
int dvm_bind(dvm_solver *s, void *f_a, void *f_b, double *moments, void *tables, void *ws);

/* dvm_upload -- copy the mesh tables and build the ghost tables (stream-ordered). */
int dvm_upload(dvm_solver *s, void *stream);

/*
 * dvm_init_maxwellian -- f := corrected discrete Maxwellian (eq. 6) of the
 * per-cell state prim[5][n_cells] = (rho, ux, uy, uz, T) (device, FP64), the
 * collision's fixed point; moments := its conserved moments.
 */
int dvm_init_maxwellian(dvm_solver *s, const double *prim, void *stream);

/*
 * dvm_step -- n_steps full steps of size dt (dt <= 0: dt from the Courant
 * number cfl, dt = cfl h_min / max_i(|xi_x| + |xi_y| + |xi_z|)), each
 * transport (eq. 2) then BGK relaxation to the corrected Maxwellian.  After
 * each step the moments buffer holds the FP64 moments of the post-transport
 * state, which the collision conserves.
 */
int dvm_step(dvm_solver *s, int32_t n_steps, double dt, double cfl, void *stream);

/*
 * dvm_global_sums -- enqueue the global FP64 conservation sums
 * sum_c V_c (rho, rho u, E) of the moments buffer (a two-level reduction in a
 * fixed order, so repeated runs agree bitwise; mass, momentum and energy are
 * the quantities the correction of eq. 6 conserves).  Asynchronous; the
 * result is read by dvm_check.
 */
int dvm_global_sums(dvm_solver *s, void *stream);

/* dvm_dt -- the step dvm_step uses for a Courant number cfl. */
int dvm_dt(const dvm_solver *s, double cfl, double *dt);

/* dvm_current_f -- device pointer of the buffer holding the current state. */
int dvm_current_f(const dvm_solver *s, void **f);

/*
 * dvm_moments -- FP64 conserved moments of the current state, out[5][n_cells]
 * (device): rho, rho ux, rho uy, rho uz, E = w sum_i (1, xi_i, |xi_i|^2/2) f_i.
 */
int dvm_moments(dvm_solver *s, double *out, void *stream);

/*
 * dvm_check -- synchronises the stream, then reports the global FP64 sums
 * sum_c V_c (rho, rho u, E) of the moments buffer and the nonphysical flag;
 * returns DVM_ERR_NONPHYSICAL if the flag is set.
 */
int dvm_check(dvm_solver *s, void *stream, dvm_diag *out);

/*
 * Step-kernel shapes (autotuning).  A shape is (threads per workgroup, waves
 * per EU variant) of the fused step kernel; each solver also chooses an XCD
 * cell grouping (runs of consecutive Morton cells kept on one XCD's L2) and plain or non-temporal
 * stores of the new state.  dvm_tune_shapes lists the shapes compiled for the
 * solver's velocity grid (at most cap; *n the total).  dvm_tune_set returns
 * DVM_ERR_UNSUPPORTED for a shape that does not exist, DVM_ERR_ARG for
 * xcd_group < 1.  The choice changes speed only: every shape computes the
 * same step (bitwise, for a given grouping of the reductions per workgroup).
 */
int dvm_tune_shapes(const dvm_solver *s, int32_t *threads, int32_t *wpe, int32_t cap, int32_t *n);
int dvm_tune_set(dvm_solver *s, int32_t threads, int32_t wpe, int32_t xcd_group, int32_t nt_store);
int dvm_tune_get(const dvm_solver *s, int32_t *threads, int32_t *wpe, int32_t *xcd_group, int32_t *nt_store);

/*
 * dvm_tune_split -- first order: step the cells that have no
 * FINER or WALL face (a level jump seen from the coarse side, or a wall) in a
 * reduced kernel and the others in a second launch of the full kernel
 * (enable = 1), or every cell in one launch (enable = 0, the default; each
 * workgroup takes the reduced code path when its cell allows it).  Both
 * compute the same step, bitwise: the reduced code only leaves out the passes
 * that such cells skip anyway.  threads_irr > 0 also
 * chooses the shape (threads per workgroup, waves-per-EU variant as listed by
 * dvm_tune_shapes) of the second launch; DVM_ERR_UNSUPPORTED if it does not
 * exist.  enable < 0 only queries; *previous (may be NULL) receives the
 * setting in use.  Without a reduced kernel for the shape chosen with
 * dvm_tune_set the step falls back to one launch.
 */
int dvm_tune_split(dvm_solver *s, int32_t enable, int32_t threads_irr, int32_t wpe_irr, int32_t *previous);

/*
 * dvm_tune -- project autotuner for one solver: time every
 * compiled step shape x XCD cell grouping {1, 8, 64, 512} x store kind (plain
 * or non-temporal) with reps trial steps on the solver's own state, keep the
 * fastest (dvm_tune_get reports it).  cache_path (may be NULL) names a text
 * file of tuned shapes, one line per key ("step", GPU architecture, N/2,
 * precision, scheme): a key found there is applied without timing
 * (*from_cache = 1, may be NULL); a timed key is added or replaced (the file
 * is rewritten through a temporary and renamed).  The trial steps read the
 * current state and write the other state buffer and the moments buffer; the
 * moments are then recomputed from the current state (within rounding of the
 * step's own values).  Synchronises.  A MUSCL solver's step kernel has one
 * shape per N (threads, waves per EU and non-temporal stores fixed): for it
 * only the XCD grouping changes what runs.  DVM_ERR_UNSUPPORTED while fluid
 * cells of a hybrid step hold no f; DVM_ERR_ARG if the cache cannot be
 * written.
 */
int dvm_tune(dvm_solver *s, const char *cache_path, int32_t reps, int32_t *from_cache, void *stream);

/*
 * dvm_tune_cache_get / dvm_tune_cache_put -- host-only access to a tuner
 * cache file (to inspect or pre-seed it): kind "step" or "batch", arch as
 * reported by the device (e.g. "gfx950"), N/2, precision (fp64 != 0), scheme;
 * shape = {threads, waves-per-EU variant, XCD cell grouping, non-temporal
 * stores}, ms the time per step the tuner measured.  *found = 0 if the key
 * is absent (shape and ms untouched).  The file is one text line per key,
 * "<kind> <arch> nh=<N/2> fp64=<0|1> scheme=<0|1> | threads=<t> wpe=<w>
 * xcd_group=<g> nt_store=<0|1> ms=<time>"; unreadable lines are ignored.
 */
int dvm_tune_cache_get(const char *path, const char *kind, const char *arch, int32_t nh, int32_t fp64,
                       int32_t scheme, int32_t shape[4], double *ms, int32_t *found);
int dvm_tune_cache_put(const char *path, const char *kind, const char *arch, int32_t nh, int32_t fp64,
                       int32_t scheme, const int32_t shape[4], double ms);

/*
 * Checkpoint and restart.
 * dvm_save -- write the solver's state to the file `path` (through
 * `path`.tmp, then renamed): a header (velocity grid, precision, scheme,
 * steps taken, root lattice, domain boundary kinds), the leaf list in cell
 * order (Morton key, level, i, j, k), f in the canonical velocity order and
 * the storage precision, the FP64 moments buffer, the hybrid step's previous
 * mask (hybrid solvers), and, if net != NULL, the network's parameter block
 * and Adam state; an FNV-1a 64-bit checksum of all of it at the end.  The
 * other state buffer serves as staging (its contents are replaced).
 * Synchronises the stream.
 * dvm_load -- read such a file into a solver built on the same leaf list,
 * velocity grid, precision and scheme (else DVM_ERR_ARG, before any device
 * write); if net != NULL the file must hold a network, which replaces net's
 * parameters and Adam state.  Stepping on after dvm_load gives bitwise the
 * steps the saved solver would have taken with the same kernel shape.
 * A checksum mismatch is reported as DVM_ERR_ARG after the state was
 * overwritten (the solver's state is then not valid).
 */
int dvm_save(dvm_solver *s, const dvm_mlp *net, const char *path, void *stream);
int dvm_load(dvm_solver *s, dvm_mlp *net, const char *path, void *stream);

/*
 * Batched steps (many independent flow instances in one graph launch).
 *
 * dvm_batch_create -- group n bound solvers (same storage precision, first
 * order) by velocity grid; inside a group the instances are
 * ordered by decreasing cost (cells x velocities) so that the largest start
 * first.  Each instance steps with its own dt = cfl h_min / max sum |xi|.
 * The solvers must outlive the batch; the batch owns host objects and the
 * recorded graphs only.
 * dvm_batch_workspace_bytes / dvm_batch_bind -- a caller-owned device block
 * (256-byte aligned) for the per-instance kernel arguments.
 * dvm_batch_step -- n_steps steps of every instance: per step one launch of
 * a recorded HIP graph holding, per velocity grid, one step kernel over the
 * cells of all its instances, then the FP64 global sums of every instance
 * (the values dvm_check reports).  The graphs are recorded at the first call
 * (and after dvm_batch_tune); a solver stepped on its own in between is
 * picked up (its buffers are re-read), DVM_ERR_WORKSPACE if a solver is not
 * uploaded.  Results are bitwise those of dvm_step on each solver with the
 * same kernel shape.
 * dvm_batch_tune -- project autotuner: for every velocity-grid group, time
 * each compiled step shape x XCD grouping {1, 8, 64} x store kind with reps
 * launches on the batch's own data and keep the fastest.  The state the
 * batch advances is unchanged (trial steps write only the next buffers; the
 * moments are recomputed from the current state afterwards).  Synchronises.
 * cache_path (may be NULL): a group whose key ("batch", GPU architecture,
 * N/2, precision) is in the tuner cache file (the format of dvm_tune) takes
 * the stored shape without timing; timed groups are added to the file.
 * dvm_batch_info -- group < 0: *n_inst = number of groups; otherwise the
 * group's velocity half-size NH (N = 2 NH), instance count, total cells and
 * chosen shape (tuned_ms: best time per launch from the last tuning, or 0).
 */
int dvm_batch_create(dvm_solver *const *solvers, int32_t n, double cfl, dvm_batch **out);
int dvm_batch_workspace_bytes(const dvm_batch *b, size_t *bytes);
int dvm_batch_bind(dvm_batch *b, void *ws);
int dvm_batch_step(dvm_batch *b, int32_t n_steps, void *stream);
int dvm_batch_tune(dvm_batch *b, int32_t reps, const char *cache_path, void *stream);
/*
 * dvm_batch_branches -- record the velocity-grid groups of a batched step as
 * parallel branches of the graph (enable = 1, the default: the groups run
 * concurrently, the global sums after all of them) or as one chain
 * (enable = 0).  The results are the same bitwise (the groups share no data).
 * enable < 0 only queries; *previous (may be NULL) receives the setting.
 */
int dvm_batch_branches(dvm_batch *b, int32_t enable, int32_t *previous);
int dvm_batch_info(const dvm_batch *b, int32_t group, int32_t *nh, int32_t *n_inst, int64_t *n_cells,
                   int32_t *threads, int32_t *wpe, int32_t *xcd_group, int32_t *nt_store, double *tuned_ms);
void dvm_destroy_batch(dvm_batch *b);

/*
 * Continuum-breakdown sensor, its training, and the kinetic/fluid hybrid step.
 *
 * Features (dvm_features; the sensor's input): per cell, from the moments
 * buffer, x[c][10] = [ln rho, u/sqrt(T) (3), ln T, lambda |grad rho|/rho,
 * lambda |grad u_b|/sqrt(T) (3), lambda |grad T|/T], lambda = tau sqrt(T),
 * gradients by central differences over face-neighbour values (the mean of
 * the four leaves of a FINER face) with centre distances h, 3h/4 (FINER),
 * 3h/2 (COARSER); a domain face uses the cell's own value.  FP32 output,
 * FP64 arithmetic.
 * Labels (dvm_labels): r[c] = |f - Mt|_2 / |Mt|_2 over the velocity nodes of
 * the current state, Mt the eq. 6 Maxwellian of the cell's own moments.
 *
 * The network 10-64-64-1 (exact GELU) lives in a caller-owned FP32 block of
 * DVM_MLP_PARAMS floats: w1[64][10], b1[64], w2[64][64], b2[64], w3[64], b3,
 * then the standardisation mean[10] and std[10] (x_std = (x - mean) / std).
 * dvm_mlp_create / dvm_mlp_workspace_bytes / dvm_mlp_bind -- host object for
 * batches of up to max_batch samples; the workspace (caller-owned, device)
 * holds the Adam moments, the gradients and per-sample scratch.  Binding
 * resets the Adam state (the caller's workspace must be zero-filled).
 * dvm_mlp_set_normalization -- mean and standard deviation of x[n][10]
 * (FP64, fixed order) into the parameter block.
 * dvm_mlp_forward -- logits z[n] of raw features x[n][10]: mode 0 FP32
 * (reference), mode 1 the matrix-core path (BF16 weights and activations,
 * FP32 accumulation; the one the sensor uses).
 * dvm_mlp_gradient -- loss and weight gradients of the class-weighted
 * binary cross-entropy mean_i w_i [softplus(z_i) - y_i z_i], w_i = pos_weight
 * for y_i = 1, else 1 (FP32 forward/backward, FP64 sums in sample order).
 * dvm_mlp_adam -- one Adam step (beta 0.9, 0.999, eps 1e-8, bias-corrected)
 * from the last gradients.  dvm_mlp_train_step = gradient + Adam.
 * dvm_mlp_buffers -- device pointers of the last gradients [DVM_MLP_WEIGHTS]
 * and loss (FP64), for inspection.
 * dvm_sensor -- mask[c] = 1 (kinetic) or 0 (fluid) for the current moments:
 * net != NULL: the network on the matrix cores, kinetic iff the logit > 0,
 * score = probability; net == NULL: the gradient-length Knudsen number
 * max(x[5..9]) against kappa, score = that number.  score may be NULL.
 *
 * dvm_hybrid_step -- n_steps steps with a frozen mask (device, n_cells
 * bytes, 1 kinetic): kinetic cells run the fused step; fluid cells advance
 * only their conserved moments U (held in the moments buffer) by the
 * half-range fluxes of the discrete velocity set, U' = U - dt/h
 * sum_faces (H_out(Mt(U)) + H_in(neighbour)), the neighbour's f when it is
 * kinetic or Mt(U_nb) when it is fluid (section 2-3 of the paper: kinetic and
 * continuum cells on one mesh).  With params.fluid_flux = DVM_FLUX_CLOSED a
 * face between two fluid cells takes instead the continuous half-range
 * integrals of both sides' Maxwellians (the same on both sides of the face,
 * so fluid cells still conserve among themselves); faces next to a kinetic
 * cell keep the discrete sums, which that cell's transport sees.  A cell that becomes kinetic starts from
 * Mt(U); one that becomes fluid keeps the moments of its f.  Cells touching
 * a non-periodic domain face stay kinetic.  Needs params.hybrid = 1 and
 * first order (DVM_ERR_UNSUPPORTED otherwise).  With every
 * cell kinetic it is dvm_step.  After hybrid steps the moments buffer is the
 * state of fluid cells (whose f rows are stale): dvm_moments then recomputes
 * kinetic cells from f and copies fluid cells' conserved moments, and must be
 * given another output than the moments buffer (DVM_ERR_ARG); dvm_step,
 * dvm_batch_create and dvm_batch_step refuse such a solver
 * (DVM_ERR_UNSUPPORTED) until a new state (dvm_init_maxwellian,
 * dvm_f_from_canonical) restores f everywhere; hybrid steps with an all-ones
 * mask continue it with every cell kinetic.
 */
#define DVM_MLP_WEIGHTS 4929
#define DVM_MLP_PARAMS 4949
int dvm_features(dvm_solver *s, float *x, void *stream);
int dvm_labels(dvm_solver *s, float *r, void *stream);
int dvm_mlp_create(int64_t max_batch, dvm_mlp **out);
int dvm_mlp_workspace_bytes(const dvm_mlp *net, size_t *bytes);
int dvm_mlp_bind(dvm_mlp *net, float *params, void *ws);
int dvm_mlp_set_normalization(dvm_mlp *net, const float *x, int64_t n, void *stream);
int dvm_mlp_forward(const dvm_mlp *net, const float *x, int64_t n, int32_t mode, float *z, void *stream);
int dvm_mlp_gradient(dvm_mlp *net, const float *x, const float *y, int64_t n, float pos_weight, void *stream);
int dvm_mlp_adam(dvm_mlp *net, float lr, void *stream);
int dvm_mlp_train_step(dvm_mlp *net, const float *x, const float *y, int64_t n, float lr, float pos_weight,
                       void *stream);
int dvm_mlp_buffers(const dvm_mlp *net, const float **grads, const double **loss);

/*
 * dvm_mlp_gradient_noalloc -- for callers that cannot allocate device memory
 * or bind a workspace (code under HIP graph capture, tight training or
 * serving loops): the loss and weight gradients of dvm_mlp_gradient, written
 * to the caller's grad[DVM_MLP_WEIGHTS] (FP32, device) and *loss (FP64,
 * device), from the parameter block params[DVM_MLP_PARAMS] (device).  No
 * network object, no workspace: the per-sample scratch lives in a static
 * device array of the library, one per GPU, sized for
 * DVM_NOALLOC_MAX_BATCH samples (about 10.4 MiB, held until the process
 * ends).  n outside [1, DVM_NOALLOC_MAX_BATCH] is DVM_ERR_WORKSPACE.  Same
 * kernels as dvm_mlp_gradient, so the same result bitwise.  Every call on a
 * GPU shares that scratch: calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialised by the caller.  Calls no
 * hipMalloc/hipFree.
 */
#define DVM_NOALLOC_MAX_BATCH 8192
int dvm_mlp_gradient_noalloc(const float *params, const float *x, const float *y, int64_t n, float pos_weight,
                             float *grad, double *loss, void *stream);
void dvm_destroy_mlp(dvm_mlp *net);
int dvm_sensor(dvm_solver *s, const dvm_mlp *net, double kappa, uint8_t *mask, float *score, void *stream);
int dvm_hybrid_step(dvm_solver *s, const uint8_t *mask, int32_t n_steps, double dt, double cfl, void *stream);

/*
 * Lattice Boltzmann subset (section 4: the LBM module as a DVM solver on a
 * minimal velocity set).  D3Q19 or D3Q27 lattice vectors c in {-1, 0, 1}^3
 * (D3Q19 without the 8 corners) on the same octree: each step is the
 * finite-volume first-order upwind transport of eq. (2) for every lattice
 * vector (periodic and outflow domain faces; a FINER face contributes the
 * mean of its four leaves), then BGK relaxation toward the second-order
 * equilibrium of section 4,
 *   f_eq = w rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 |u|^2)   (cs^2 = 1/3),
 * weights by |c|^2 = 0, 1, 2, 3: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27,
 * 1/54, 1/216; exponential (f_eq + (f* - f_eq) e^{-dt/tau}) or explicit
 * Euler relaxation.  rho = sum f, rho u = sum c f (mass and momentum are
 * conserved; the model is isothermal).
 * Buffers (caller-owned, 256-byte aligned, sizes from dvm_lbm_buffer_sizes):
 * two state buffers f[q][n_cells] (population-major, storage precision),
 * moments [5][n_cells] FP64, tables (32-byte cell records and the FINER-face
 * leaf lists), workspace (reduction partials, sums, flag).
 * dvm_lbm_create -- DVM_ERR_UNSUPPORTED if the mesh has inflow or wall faces.
 * dvm_lbm_init -- f := f_eq of prim[4][n_cells] (rho, ux, uy, uz; device FP64).
 * dvm_lbm_step -- dt <= 0: dt = cfl h_min / max_i (|c_x| + |c_y| + |c_z|)
 * (2 for D3Q19, 3 for D3Q27).
 * dvm_lbm_moments -- out[5][n_cells] = (rho, rho u, sum |c|^2 f / 2).
 * dvm_lbm_check -- synchronises; global sums sum_c V_c (moments) and the flag
 * (rho <= 0 or NaN).
 * dvm_lbm_get_f / dvm_lbm_set_f -- the current state as [n_cells][27] in the
 * canonical order of the 3^3 grid (kx*9 + ky*3 + kz, c = k - 1), storage
 * precision, corners zero for D3Q19.
 */
typedef struct dvm_lbm dvm_lbm;
typedef struct {
    int32_t q;                /* 19 or 27 */
    int32_t precision;        /* DVM_PREC_* */
    int32_t collision;        /* DVM_COLL_EXP or DVM_COLL_EULER */
    double tau;               /* relaxation time */
} dvm_lbm_params;
int dvm_lbm_create(const dvm_mesh *m, const dvm_lbm_params *p, dvm_lbm **out);
int dvm_lbm_buffer_sizes(const dvm_lbm *s, dvm_sizes *out);
int dvm_lbm_bind(dvm_lbm *s, void *f_a, void *f_b, double *moments, void *tables, void *ws);
int dvm_lbm_upload(dvm_lbm *s, void *stream);
int dvm_lbm_init(dvm_lbm *s, const double *prim, void *stream);
int dvm_lbm_dt(const dvm_lbm *s, double cfl, double *dt);
int dvm_lbm_step(dvm_lbm *s, int32_t n_steps, double dt, double cfl, void *stream);
int dvm_lbm_moments(dvm_lbm *s, double *out, void *stream);
int dvm_lbm_check(dvm_lbm *s, void *stream, dvm_diag *out);
int dvm_lbm_get_f(const dvm_lbm *s, void *out, void *stream);
int dvm_lbm_set_f(dvm_lbm *s, const void *in, void *stream);
int dvm_lbm_current_f(const dvm_lbm *s, void **f);
void dvm_destroy_lbm(dvm_lbm *s);

/*
 * On-device mesh adaptation (section 3.1 step 4: the cell order and the
 * stencil are rebuilt each time the mesh changes; section 3.3: on the device).
 * Meshes without solid leaves.  The library allocates nothing: the caller
 * passes a device workspace of dvm_adapt_workspace_bytes(max_leaves) bytes.
 * dvm_adapt_leaves -- from the solver's mesh and per-cell flags (device,
 * int8: +1 refine into 8 children, -1 coarsen: a complete set of 8 sibling
 * leaves that all ask is replaced by their parent, 0 keep), then the 2:1
 * closure over faces, edges and corners (section 2.1; more leaves are
 * refined as needed): the new leaves in Morton order into level_out[cap],
 * ijk_out[cap][3] (device); *n_out (host) their number.  DVM_ERR_WORKSPACE if
 * more than cap (then *n_out is the number needed).  Synchronises.
 * dvm_adapt_mesh -- the mesh record of an adapted leaf list (device arrays
 * from dvm_adapt_leaves, n leaves): domain and boundary kinds of `old`, the
 * leaf list copied to the host (13 bytes per leaf, for the solver's sizes and
 * checkpoints) and NO host face tables: each solver on it gets its tables from
 * dvm_adapt_tables.  dvm_mesh_export refuses to export its tables and the LBM
 * path refuses it; destroy with dvm_destroy_mesh.  Synchronises.
 * dvm_adapt_tables -- the face tables of a solver on the adapted leaf list,
 * built on the device from the device leaf list (Morton order) into the
 * solver's bound tables buffer (the same records the host builder makes), and
 * the step's selection list of regular cells; the mesh's face counts
 * (dvm_mesh_info) are set from them.  Call after dvm_upload: a solver on a
 * dvm_adapt_mesh mesh is not ready (DVM_ERR_WORKSPACE "call dvm_upload first"
 * from every other call) until this returns DVM_OK.  On a solver of a mesh
 * made by dvm_create_mesh of the same list it rewrites the same bytes.
 * DVM_ERR_UNBALANCED if the list is not a 2:1-balanced partition.
 * Synchronises.
 * dvm_adapt_remap -- the current state of `to` from the current state of
 * `from` (same domain, velocity grid and precision): a new cell inside an old
 * leaf takes its row, a new cell covering several old leaves their
 * volume-weighted mean (FP64 sums in key order), so mass, momentum and energy
 * are conserved; then `to`'s moments are recomputed.  Workspace: the two leaf
 * lists and their keys (dvm_adapt_workspace_bytes(n_from + n_to) is enough).
 */
int dvm_adapt_workspace_bytes(int64_t max_leaves, size_t *bytes);
int dvm_adapt_leaves(const dvm_solver *s, const int8_t *flags, int64_t cap, uint8_t *level_out, int32_t *ijk_out,
                     int64_t *n_out, void *ws, size_t ws_bytes, void *stream);
int dvm_adapt_mesh(const dvm_mesh *old, const uint8_t *level, const int32_t *ijk, int64_t n, dvm_mesh **out,
                   void *stream);
int dvm_adapt_tables(dvm_solver *s, const uint8_t *level, const int32_t *ijk, void *ws, size_t ws_bytes,
                     void *stream);
int dvm_adapt_remap(const dvm_solver *from, dvm_solver *to, void *ws, size_t ws_bytes, void *stream);

/* canonical <-> internal velocity order of one state buffer [n_cells][N^3] */
int dvm_f_to_canonical(const dvm_solver *s, const void *f_internal, void *f_canon, void *stream);
int dvm_f_from_canonical(dvm_solver *s, const void *f_canon, void *f_internal, void *stream);

void dvm_destroy_solver(dvm_solver *s);

#ifdef __cplusplus
}
#endif
#endif /* DVM_H */
