// solver_impl.h -- the solver object shared by the host sources (solver.cpp,
// batch.cpp).  Holds no device memory of its own: every buffer is bound by
// the caller (dvm_bind).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"
#include "kernels.h"

namespace dvm {

constexpr int kPartials = 1024;  // blocks of the first global-sum stage

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline int hip_fail(hipError_t e, const char *what) {
    return fail(DVM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

inline hipStream_t S(void *stream) { return static_cast<hipStream_t>(stream); }

}  // namespace dvm

struct dvm_solver {
    const dvm_mesh *m = nullptr;
    dvm_params p{};
    bool fp64 = false;
    int nh = 0;
    int64_t nv = 0;
    int64_t n = 0;
    dvm::VelGrid g{};
    dvm::StepConfig cfg{};
    size_t f_bytes = 0, mom_bytes = 0, tab_bytes = 0, ws_bytes = 0;
    // workspace sections (byte offsets)
    size_t off_gin = 0, off_m1 = 0, off_den = 0, off_flag = 0, off_part = 0, off_sums = 0;
    size_t off_kor = 0;          // Korobov collision: trial table [p][NV] (64-bit entries)
    std::vector<uint64_t> kor_host;
    int64_t kor_p = 0, kor_a = 0;
    size_t off_hyb = 0;          // hybrid: masks (effective, previous, row flags) [n], flux sums [n][66],
                                 // interface face fluxes [n][6][5]
    bool hybrid = false;
    bool hybrid_fluid = false;   // fluid cells may exist (their f is stale)
    bool muscl = false;
    void *f[2] = {nullptr, nullptr};
    int cur = 0;
    double *mom = nullptr;
    dvm::DevCell *tables = nullptr;
    char *ws = nullptr;
    bool uploaded = false;
    bool tables_pending = false;  // uploaded except the face tables of a device-table mesh
    int64_t steps = 0;
    bool has_inflow = false, has_wall = false;
    int n_cu = 0;                  // compute units of the bound device
    // first order: optionally step the cells without FINER or
    // WALL faces ("regular") in a reduced kernel and the others in a second
    // launch (off by default: one launch takes the reduced code path per cell
    // and keeps Morton locality between the two kinds)
    bool split = false;
    int64_t n_reg = 0;             // regular cells: the first n_reg entries of the selection list
    size_t off_sel = 0;            // selection list [n] (regular cells, then the others; Morton order)
    std::vector<uint32_t> sel_host;
    dvm::StepConfig cfg_irr{};     // shape of the launch over the other cells

    void *gin() const { return ws + off_gin; }
    void *m1() const { return ws + off_m1; }
    const uint64_t *kor() const { return reinterpret_cast<const uint64_t *>(ws + off_kor); }
    bool korobov() const { return p.collision == DVM_COLL_KOROBOV; }
    double *den() const { return reinterpret_cast<double *>(ws + off_den); }
    int *flag() const { return reinterpret_cast<int *>(ws + off_flag); }
    double *partials() const { return reinterpret_cast<double *>(ws + off_part); }
    double *sums() const { return reinterpret_cast<double *>(ws + off_sums); }
    const uint32_t *sel() const { return reinterpret_cast<const uint32_t *>(ws + off_sel); }
};

// The sensor network: host object over a caller-owned parameter block and
// workspace (Adam moments, gradients, per-sample scratch).
struct dvm_mlp {
    int64_t max_batch = 0;
    float *params = nullptr;
    char *ws = nullptr;
    size_t off_m = 0, off_v = 0, off_grad = 0, off_rec = 0, off_lpart = 0, off_loss = 0, ws_bytes = 0;
    int64_t t = 0;  // Adam step count

    float *m() const { return reinterpret_cast<float *>(ws + off_m); }
    float *v() const { return reinterpret_cast<float *>(ws + off_v); }
    float *grad() const { return reinterpret_cast<float *>(ws + off_grad); }
    float *rec() const { return reinterpret_cast<float *>(ws + off_rec); }
    double *lpart() const { return reinterpret_cast<double *>(ws + off_lpart); }
    double *loss() const { return reinterpret_cast<double *>(ws + off_loss); }
};

namespace dvm {
// Kernel arguments of one fused step of size dt (f_in / f_out left NULL).
StepArgs solver_step_args(const dvm_solver *s, double dt);
double solver_max_speed_sum(const dvm_solver *s);
// f[cur] was replaced from outside the step (a remap): records, hybrid masks
// and the moments buffer describe the new state
hipError_t solver_state_replaced(dvm_solver *s, hipStream_t st);
// every cell kinetic again (a fresh state); no-op without the hybrid workspace
hipError_t solver_reset_hybrid(dvm_solver *s, hipStream_t st);
// fluid cells of the last hybrid step: out[5][n] := their conserved moments
hipError_t solver_fluid_moments(const dvm_solver *s, double *out, hipStream_t st);
// the hybrid step's mask of the previous step [n] (NULL without the hybrid workspace)
uint8_t *solver_hybrid_prev(const dvm_solver *s);

// Tuner cache: one line per (kind, GPU architecture, N/2, precision, scheme)
// with the chosen kernel shape.  kind is "step" (one solver) or "batch".
struct TuneKey {
    const char *kind;
    int nh;
    int fp64;
    int scheme;
};
// architecture name of the current device (e.g. "gfx950"), "" on failure
std::string device_arch();
// true and *cfg (threads, wpe, xcd_group, nt_store) if the cache holds the key
bool tune_cache_get(const char *path, const TuneKey &k, StepConfig *cfg, double *ms);
// add or replace the key's line; DVM_OK or a DVM_ERR_* (with the error text set)
int tune_cache_put(const char *path, const TuneKey &k, const StepConfig &cfg, double ms);
// the same for a named architecture
bool tune_cache_get_arch(const char *path, const TuneKey &k, const std::string &arch, StepConfig *cfg, double *ms);
int tune_cache_put_arch(const char *path, const TuneKey &k, const std::string &arch, const StepConfig &cfg,
                        double ms);
}  // namespace dvm
