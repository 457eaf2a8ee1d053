// kernels.h -- launch interface between the solver host code and the HIP
// kernels (kernels.hip).  Plain structs passed by value as kernel arguments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.h"

namespace dvm {

struct VelGrid {
    int nh;          // N/2 nodes per half axis
    double dv[3];    // node spacing per axis
    double w;        // dv[0]*dv[1]*dv[2]
};

struct StepArgs {
    const void *f_in;
    void *f_out;
    double *mom;             // [5][n_cells]
    const DevCell *cells;
    const void *ghost_in;    // inflow Maxwellian, internal velocity order
    const void *wall_m1;     // unit-density wall Maxwellian
    const double *wall_den;  // [6] sum_{xi.n<0} |xi.n| M1 per face direction
    int *flag;               // nonphysical flag
    int64_t n_cells;
    double dt;
    double h0;
    VelGrid g;
    int collision;           // DVM_COLL_*
    int tau_mode;            // DVM_TAU_*
    double tau_or_kn;
    int xcd_log2;            // runs of 2^xcd_log2 consecutive cells kept on one XCD
    int muscl;               // 1: MUSCL-minmod transport (reconstructed in the step), 0: first order
    const uint32_t *sel;     // the cells this launch steps, one per workgroup (NULL: 0 .. n_cells-1)
    int64_t n_sel;           // their number (used when sel is set)
};

struct InitArgs {
    const double *prim;      // [5][n] rho, ux, uy, uz, T; NULL: use prim0
    double prim0[5];
    void *f_out;             // [n][NV] internal order
    double *mom;             // [5][n] or NULL
    int *flag;
    int64_t n;
    VelGrid g;
};

// Kernel-configuration choice for one (precision, N) pair.
struct StepConfig {
    int threads;     // workgroup size
    int xcd_group;   // consecutive cells kept on one XCD
    int nt_store;    // non-temporal stores of the new state
    int wpe;         // waves-per-EU variant (0: the first listed for this shape)
    int regular;     // 1: the launch holds only cells without FINER or WALL faces (reduced kernel)
};

// All return hipError_t of the launch (hipErrorInvalidValue: no kernel for N).
hipError_t launch_step(bool fp64, const StepArgs &a, const StepConfig &cfg, hipStream_t st);
hipError_t launch_init(bool fp64, const InitArgs &a, hipStream_t st);
hipError_t launch_moments(bool fp64, const void *f, double *out, int64_t n, const VelGrid &g, hipStream_t st);
hipError_t launch_wall_den(bool fp64, const void *m1, double *den, const VelGrid &g, hipStream_t st);
hipError_t launch_global_sums(const double *mom, const DevCell *cells, int64_t n, double h0, double *partials,
                              int n_part, double *out, hipStream_t st);
hipError_t launch_to_canonical(bool fp64, bool to_canon, const void *src, void *dst, int64_t n, int nh,
                               hipStream_t st);
bool have_kernel(int nh, int threads, int wpe);
// a reduced kernel (cells without FINER or WALL faces) exists for this shape
bool have_regular_kernel(int nh, int threads, int wpe);
int list_kernels(int nh, int *threads, int *wpe, int cap);
int default_threads(bool fp64, int nh);

// Batched steps (batch.cpp): instance arguments in device memory.
struct SumArgs {
    const double *mom;       // [5][n]
    const DevCell *cells;
    int64_t n;
    double h0;
    double *partials;        // [kPartials][5]
    double *out;             // [5]
};
hipError_t launch_step_batch(bool fp64, const StepArgs *inst, const uint32_t *wg_end, int n_inst, uint32_t total_wg,
                             int nh, const StepConfig &cfg, hipStream_t st);
hipError_t launch_global_sums_batch(const SumArgs *inst, int n_inst, int n_part, hipStream_t st);

// Sensor, training and hybrid step (sensor.hip).
struct SensorArgsPub {
    const double *mom;
    const DevCell *cells;
    int64_t n;
    double h0;
    int tau_mode;
    double tau_or_kn;
};
struct HybArgsPub {
    const uint8_t *mask;
    uint8_t *prev;
    uint8_t *rows;
    double *flux;
    double *face;
    int32_t closed;  // fluid-fluid faces: continuous half-range integrals
    int32_t pad;
};
constexpr int kMlpParams = 4949, kMlpWeights = 4929, kMlpRecord = 331, kFluxRecord = 71, kFaceRecord = 30;
hipError_t launch_features(const SensorArgsPub &a, float *x, hipStream_t st);
hipError_t launch_labels(bool fp64, const void *f, float *r, int64_t n, const VelGrid &g, hipStream_t st);
hipError_t launch_mlp_forward(const float *params, const float *x, int64_t n, int mode, float *z, hipStream_t st);
hipError_t launch_sensor(const SensorArgsPub &a, const float *params, double kappa, uint8_t *mask, float *score,
                         hipStream_t st);
hipError_t launch_train(const float *params, const float *x, const float *y, int64_t n, float pos_weight,
                        float *rec, double *loss_part, float *grad, double *loss, hipStream_t st);
hipError_t launch_adam(float *params, float *m, float *v, const float *grad, float lr, float c1, float c2,
                       hipStream_t st);
// launch_train with its scratch in a static device array (no allocation)
constexpr int64_t kNoAllocMaxBatch = 8192;
hipError_t launch_train_noalloc(const float *params, const float *x, const float *y, int64_t n, float pos_weight,
                                float *grad, double *loss, hipStream_t st);
hipError_t launch_norm_stats(const float *x, int64_t n, float *params, hipStream_t st);
hipError_t launch_mask_eff(const uint8_t *in, uint8_t *out, const DevCell *cells, int64_t n, hipStream_t st);
hipError_t launch_hybrid(bool fp64, const StepArgs &a, const HybArgsPub &h, hipStream_t st);
hipError_t launch_fluid_moments(const uint8_t *mask, const double *mom, double *out, int64_t n, hipStream_t st);

// Boltzmann collision integral on Korobov nodes (korobov.hip / korobov.cpp).
struct KorArgs {
    void *f;                 // [n_cells][NV] post-transport state, updated in place
    const uint64_t *table;   // [p][NV] entries j | l << 16 | m << 32 | n << 48 (internal indices; 0xFFFF:
                             // no gain; n = |k_j - k_i|^2 in node units)
    int64_t n_cells;
    int p;
    double w0;               // V_box / p
    double dt_kn;            // dt / Kn
    double vmax;             // half width of the velocity grid (basis scale)
    VelGrid g;
    int *flag;               // raised if a conservation system is singular
};
hipError_t launch_korobov(bool fp64, const KorArgs &a, hipStream_t st);
bool korobov_supported(int nh);
int64_t korobov_generator(int64_t p);
void korobov_tables(int n, double vmax, int64_t p, int64_t a, std::vector<int32_t> &J, std::vector<int32_t> &L,
                    std::vector<int32_t> &M);
void korobov_device_table(int nh, const std::vector<int32_t> &J, const std::vector<int32_t> &L,
                          const std::vector<int32_t> &M, int64_t p, std::vector<uint64_t> &out);

// Lattice Boltzmann subset (lbm.hip / lbm.cpp).
struct LbmCell {        // 32 bytes per cell
    int32_t nb[6];      // the neighbour of a SAME or COARSER face (face order -x, +x, -y, +y, -z, +z)
    uint32_t meta;      // face kinds, 3 bits per face (bits 0..17); level in bits 24..31
    int32_t fine;       // first of the cell's FINER-face tuples (4 cells each, face order) in the fine list
};
static_assert(sizeof(LbmCell) == 32, "LbmCell must stay 32 bytes");
struct LbmArgs {
    const void *f_in;   // [Q][n]
    void *f_out;
    const LbmCell *cells;
    const int32_t *fine;
    int64_t n;
    double dt, h0;
    double relax;       // exp(-dt/tau) (exponential) or dt/tau (explicit Euler)
    int euler;
    int *flag;
    int xcd_log2;       // workgroups of 256 cells go to the XCDs in runs of 2^xcd_log2
};
hipError_t launch_lbm_step(int q, bool fp64, const LbmArgs &a, hipStream_t st);
hipError_t launch_lbm_moments(int q, bool fp64, const void *f, const LbmCell *cells, int64_t n, double h0,
                              double *mom, double *partials, double *sums, hipStream_t st);
hipError_t launch_lbm_init(int q, bool fp64, const double *prim, void *f, int64_t n, int *flag, hipStream_t st);
hipError_t launch_lbm_canon(int q, bool fp64, const void *src, void *dst, int64_t n, bool to_canon, hipStream_t st);


// per-precision instantiations (kernels_f32.hip, kernels_f64.hip)
#define DVM_DECLARE_PREC(SUF)                                                                            \
    hipError_t launch_step_##SUF(const StepArgs &a, const StepConfig &cfg, hipStream_t st);              \
    hipError_t launch_step_batch_##SUF(const StepArgs *inst, const uint32_t *wg_end, int n_inst,         \
                                       uint32_t total_wg, int nh, const StepConfig &cfg, hipStream_t st); \
    hipError_t launch_init_##SUF(const InitArgs &a, hipStream_t st);                                     \
    hipError_t launch_moments_##SUF(const void *f, double *out, int64_t n, const VelGrid &g, hipStream_t st); \
    hipError_t launch_wall_den_##SUF(const void *m1, double *den, const VelGrid &g, hipStream_t st);
DVM_DECLARE_PREC(f32)
DVM_DECLARE_PREC(f64)
#undef DVM_DECLARE_PREC

}  // namespace dvm
