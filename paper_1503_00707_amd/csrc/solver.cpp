// solver.cpp -- host side of the solver: argument checks, buffer layout,
// kernel launches on the caller's stream.  Holds no device memory of its own:
// every buffer is bound by the caller (dvm_bind).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "solver_impl.h"

using namespace dvm;

namespace {
// two launches (reduced kernel over the regular cells, full kernel over the
// rest) instead of one: first order, kernels compiled
bool use_split(const dvm_solver *s) {
    return s->split && !s->muscl && s->n_reg > 0 && have_regular_kernel(s->nh, s->cfg.threads, s->cfg.wpe) &&
           have_kernel(s->nh, s->cfg_irr.threads, s->cfg_irr.wpe);
}
}  // namespace

StepArgs dvm::solver_step_args(const dvm_solver *s, double dt) {
    StepArgs a{};
    a.mom = s->mom;
    a.cells = s->tables;
    a.ghost_in = s->gin();
    a.wall_m1 = s->m1();
    a.wall_den = s->den();
    a.flag = s->flag();
    a.n_cells = s->n;
    a.dt = dt;
    a.h0 = s->m->h0;
    a.g = s->g;
    // the Korobov collision runs as its own kernel after a transport-only step
    a.collision = s->korobov() ? DVM_COLL_OFF : s->p.collision;
    a.tau_mode = s->p.tau_mode;
    a.tau_or_kn = s->p.tau_or_kn;
    a.xcd_log2 = 0;
    while ((1 << (a.xcd_log2 + 1)) <= s->cfg.xcd_group) ++a.xcd_log2;
    a.muscl = s->muscl ? 1 : 0;
    return a;
}

hipError_t dvm::solver_state_replaced(dvm_solver *s, hipStream_t st) {
    hipError_t e = solver_reset_hybrid(s, st);
    if (e == hipSuccess) e = launch_moments(s->fp64, s->f[s->cur], s->mom, s->n, s->g, st);
    s->hybrid_fluid = false;
    return e;
}

double dvm::solver_max_speed_sum(const dvm_solver *s) {
    double r = 0.0;
    for (int b = 0; b < 3; ++b) r += (s->nh - 0.5) * s->g.dv[b];
    return r;
}

extern "C" {

int dvm_create_solver(const dvm_mesh *m, const dvm_params *p, dvm_solver **out) {
    clear_error();
    if (!m || !p || !out) return fail(DVM_ERR_ARG, "null argument");
    *out = nullptr;
    if (p->nv < 2 || p->nv % 2) return fail(DVM_ERR_UNSUPPORTED, "nv = %d: the device path needs an even N", p->nv);
    for (int b = 0; b < 3; ++b)
        if (!(p->vmax[b] > 0)) return fail(DVM_ERR_ARG, "vmax[%d] must be > 0", b);
    if (p->precision != DVM_PREC_FP64 && p->precision != DVM_PREC_FP32) return fail(DVM_ERR_ARG, "bad precision");
    if (p->scheme != DVM_SCHEME_UPWIND1 && p->scheme != DVM_SCHEME_MUSCL) return fail(DVM_ERR_ARG, "bad scheme");
    if (p->collision < DVM_COLL_EXP || p->collision > DVM_COLL_KOROBOV) return fail(DVM_ERR_ARG, "bad collision mode");
    if (p->tau_mode != DVM_TAU_CONST && p->tau_mode != DVM_TAU_HS) return fail(DVM_ERR_ARG, "bad tau mode");
    if (p->fluid_flux != DVM_FLUX_GRID && p->fluid_flux != DVM_FLUX_CLOSED) return fail(DVM_ERR_ARG, "bad fluid_flux");
    if (p->collision != DVM_COLL_OFF && !(p->tau_or_kn > 0)) return fail(DVM_ERR_ARG, "tau_or_kn must be > 0");
    const bool fp64 = p->precision == DVM_PREC_FP64;
    const int nh = p->nv / 2;
    const int thr = default_threads(fp64, nh);
    if (!thr) return fail(DVM_ERR_UNSUPPORTED, "no device kernel for N = %d (have 4, 8, 12, 16, 24)", p->nv);
    int64_t kor_a = 0;
    if (p->collision == DVM_COLL_KOROBOV) {
        if (!korobov_supported(nh)) return fail(DVM_ERR_UNSUPPORTED, "Korobov collision kernel for N = 4, 8, 12 only");
        if (p->hybrid) return fail(DVM_ERR_UNSUPPORTED, "the hybrid step relaxes with BGK");
        if (p->vmax[0] != p->vmax[1] || p->vmax[0] != p->vmax[2])
            return fail(DVM_ERR_UNSUPPORTED, "Korobov collision on a cubic velocity box only");
        const int64_t gen = korobov_generator(p->korobov_p);
        if (gen < 0) return fail(DVM_ERR_ARG, "korobov_p = %d must be a prime in [5, 2^31)", p->korobov_p);
        kor_a = p->korobov_a ? p->korobov_a : gen;
        if (kor_a < 1 || kor_a >= p->korobov_p) return fail(DVM_ERR_ARG, "korobov_a must be in [1, p)");
    }
    dvm_solver *s = new (std::nothrow) dvm_solver();
    if (!s) return fail(DVM_ERR_ARG, "out of host memory");
    s->m = m;
    s->p = *p;
    s->fp64 = fp64;
    s->nh = nh;
    s->nv = int64_t(p->nv) * p->nv * p->nv;
    s->n = int64_t(m->cells.size());
    s->g.nh = nh;
    s->g.w = 1.0;
    for (int b = 0; b < 3; ++b) {
        s->g.dv[b] = 2.0 * p->vmax[b] / p->nv;
        s->g.w *= s->g.dv[b];
    }
    // measured defaults per (precision, N); dvm_tune_set overrides them
    s->cfg.threads = thr;
    s->cfg.xcd_group = 1;
    s->cfg.nt_store = 0;
    s->cfg.wpe = 0;
    if (nh == 12 && !fp64) {
        s->cfg.threads = 192;
        s->cfg.wpe = 31;
        s->cfg.xcd_group = 512;
        s->cfg.nt_store = 1;
    }
    if ((nh == 6 || nh == 8) && !fp64) {
        // 12^3 and 16^3: per-cell fixed work (reductions, the Maxwellian
        // system) dominates, and two waves per cell keep more cells in flight
        s->cfg.threads = 128;
        s->cfg.wpe = nh == 6 ? 60 : 50;
        s->cfg.xcd_group = 64;
        s->cfg.nt_store = 1;
    }
    if (nh == 12 && fp64) {
        s->cfg.threads = 576;
        s->cfg.wpe = 30;
        s->cfg.xcd_group = 64;
        s->cfg.nt_store = 1;
    }
    if (m->device_tables) {
        // no solid leaves: domain faces are the only INFLOW / WALL faces
        for (int f = 0; f < 6; ++f) {
            s->has_inflow |= m->bc[f] == DVM_BC_INFLOW;
            s->has_wall |= m->bc[f] == DVM_BC_WALL;
        }
    } else {
        s->has_inflow = m->n_faces[DVM_FACE_INFLOW] > 0;
        s->has_wall = m->n_faces[DVM_FACE_WALL] > 0;
    }
    const size_t fs = fp64 ? 8 : 4;
    s->f_bytes = align256(size_t(s->n) * size_t(s->nv) * fs);
    s->mom_bytes = align256(size_t(5) * size_t(s->n) * 8);
    s->tab_bytes = align256(size_t(s->n) * sizeof(DevCell));
    size_t o = 0;
    s->off_gin = o;  o += align256(size_t(s->nv) * fs);
    s->off_m1 = o;   o += align256(size_t(s->nv) * fs);
    s->off_den = o;  o += align256(6 * 8);
    s->off_flag = o; o += 256;
    s->off_part = o; o += align256(size_t(kPartials) * 5 * 8);
    s->off_sums = o; o += 256;
    s->muscl = p->scheme == DVM_SCHEME_MUSCL;
    s->off_kor = o;
    if (p->collision == DVM_COLL_KOROBOV) {
        s->kor_p = p->korobov_p;
        s->kor_a = kor_a;
        std::vector<int32_t> J, L, M;
        korobov_tables(p->nv, p->vmax[0], s->kor_p, s->kor_a, J, L, M);
        korobov_device_table(nh, J, L, M, s->kor_p, s->kor_host);
        o += align256(s->kor_host.size() * sizeof(uint64_t));
    }
    s->hybrid = p->hybrid != 0;
    s->off_hyb = o;
    if (s->hybrid)
        o += 3 * align256(size_t(s->n)) + align256(size_t(s->n) * kFluxRecord * 8) +
             align256(size_t(s->n) * kFaceRecord * 8);
    // selection list: regular cells (no FINER or WALL face) first, then the rest
    s->off_sel = o;  o += align256(size_t(s->n) * 4);
    if (!m->device_tables) s->sel_host.reserve(size_t(s->n));
    for (int pass = 0; pass < 2 && !m->device_tables; ++pass)
        for (int64_t c = 0; c < s->n; ++c) {
            const DevCell &d = m->table[size_t(c)];
            bool irregular = false;
            for (int f = 0; f < 6; ++f) irregular |= d.type[f] == DVM_FACE_FINER || d.type[f] == DVM_FACE_WALL;
            if (irregular == (pass == 1)) s->sel_host.push_back(uint32_t(c));
            if (pass == 0 && !irregular) ++s->n_reg;
        }
    s->cfg_irr = s->cfg;
    s->ws_bytes = o;
    *out = s;
    return DVM_OK;
}

int dvm_buffer_sizes(const dvm_solver *s, dvm_sizes *out) {
    clear_error();
    if (!s || !out) return fail(DVM_ERR_ARG, "null argument");
    out->f_bytes = s->f_bytes;
    out->moments_bytes = s->mom_bytes;
    out->tables_bytes = s->tab_bytes;
    out->ws_bytes = s->ws_bytes;
    out->n_cells = s->n;
    out->nv_total = s->nv;
    return DVM_OK;
}

int dvm_bind(dvm_solver *s, void *f_a, void *f_b, double *moments, void *tables, void *ws) {
    clear_error();
    if (!s) return fail(DVM_ERR_ARG, "null solver");
    void *ptrs[5] = {f_a, f_b, moments, tables, ws};
    for (void *q : ptrs) {
        if (!q) return fail(DVM_ERR_WORKSPACE, "a buffer is NULL");
        if (reinterpret_cast<uintptr_t>(q) & 255) return fail(DVM_ERR_ARG, "buffers must be 256-byte aligned");
    }
    if (f_a == f_b) return fail(DVM_ERR_ARG, "the two state buffers must differ");
    s->f[0] = f_a;
    s->f[1] = f_b;
    s->cur = 0;
    s->mom = moments;
    s->tables = static_cast<DevCell *>(tables);
    s->ws = static_cast<char *>(ws);
    s->uploaded = false;
    s->tables_pending = false;
    s->steps = 0;
    return DVM_OK;
}

int dvm_upload(dvm_solver *s, void *stream) {
    clear_error();
    if (!s || !s->ws) return fail(DVM_ERR_WORKSPACE, "solver not bound");
    hipStream_t st = S(stream);
    const bool dev_tab = s->m->device_tables;
    hipError_t e = hipSuccess;
    if (!dev_tab) {
        e = hipMemcpyAsync(s->tables, s->m->table.data(), s->m->table.size() * sizeof(DevCell),
                           hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(tables)");
    }
    e = hipMemsetAsync(s->ws, 0, s->ws_bytes, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(ws)");
    if (!dev_tab) {
        e = hipMemcpyAsync(s->ws + s->off_sel, s->sel_host.data(), s->sel_host.size() * 4, hipMemcpyHostToDevice,
                           st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(selection)");
    }
    InitArgs a{};
    a.prim = nullptr;
    a.n = 1;
    a.g = s->g;
    a.flag = s->flag();
    a.mom = nullptr;
    if (s->has_inflow) {
        for (int k = 0; k < 5; ++k) a.prim0[k] = s->p.inflow[k];
        a.f_out = s->gin();
        e = launch_init(s->fp64, a, st);
        if (e != hipSuccess) return hip_fail(e, "inflow ghost");
    }
    if (s->has_wall) {
        const double pw[5] = {1.0, 0.0, 0.0, 0.0, s->p.t_wall};
        for (int k = 0; k < 5; ++k) a.prim0[k] = pw[k];
        a.f_out = s->m1();
        e = launch_init(s->fp64, a, st);
        if (e != hipSuccess) return hip_fail(e, "wall Maxwellian");
        e = launch_wall_den(s->fp64, s->m1(), s->den(), s->g, st);
        if (e != hipSuccess) return hip_fail(e, "wall denominators");
    }
    if (s->korobov()) {
        e = hipMemcpyAsync(s->ws + s->off_kor, s->kor_host.data(), s->kor_host.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "Korobov table");
    }
    e = solver_reset_hybrid(s, st);
    if (e != hipSuccess) return hip_fail(e, "hybrid masks");
    s->hybrid_fluid = false;
    {
        int dev = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "device attributes");
    }
    // the host table must stay valid until the copy has been consumed
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    // a device-table mesh is ready once dvm_adapt_tables has built its tables
    s->uploaded = !dev_tab;
    s->tables_pending = dev_tab;
    return DVM_OK;
}

int dvm_init_maxwellian(dvm_solver *s, const double *prim, void *stream) {
    clear_error();
    if (!s || !prim) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    InitArgs a{};
    a.prim = prim;
    a.n = s->n;
    a.g = s->g;
    a.flag = s->flag();
    a.mom = s->mom;
    s->cur = 0;
    a.f_out = s->f[0];
    hipError_t e = launch_init(s->fp64, a, S(stream));
    if (e != hipSuccess) return hip_fail(e, "init");
    e = solver_reset_hybrid(s, S(stream));
    if (e != hipSuccess) return hip_fail(e, "hybrid masks");
    s->hybrid_fluid = false;
    s->steps = 0;
    return DVM_OK;
}

int dvm_dt(const dvm_solver *s, double cfl, double *dt) {
    clear_error();
    if (!s || !dt) return fail(DVM_ERR_ARG, "null argument");
    if (!(cfl > 0)) return fail(DVM_ERR_ARG, "cfl must be > 0");
    *dt = cfl * s->m->h_min / solver_max_speed_sum(s);
    return DVM_OK;
}

int dvm_step(dvm_solver *s, int32_t n_steps, double dt, double cfl, void *stream) {
    clear_error();
    if (!s) return fail(DVM_ERR_ARG, "null solver");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    if (n_steps < 0) return fail(DVM_ERR_ARG, "n_steps < 0");
    if (s->hybrid_fluid)
        return fail(DVM_ERR_UNSUPPORTED, "fluid cells hold no f: continue with dvm_hybrid_step (an all-ones mask "
                                         "turns every cell kinetic)");
    if (!(dt > 0)) {
        int rc = dvm_dt(s, cfl, &dt);
        if (rc) return rc;
    }
    StepArgs a = solver_step_args(s, dt);
    hipStream_t st = S(stream);
    hipError_t e = hipSuccess;
    for (int it = 0; it < n_steps; ++it) {
        a.f_in = s->f[s->cur];
        a.f_out = s->f[s->cur ^ 1];
        if (use_split(s)) {
            StepArgs ar = a;
            ar.sel = s->sel();
            ar.n_sel = s->n_reg;
            StepConfig cr = s->cfg;
            cr.regular = 1;
            e = s->n_reg > 0 ? launch_step(s->fp64, ar, cr, st) : hipSuccess;
            if (e == hipSuccess && s->n > s->n_reg) {
                StepArgs ai = a;
                ai.sel = s->sel() + s->n_reg;
                ai.n_sel = s->n - s->n_reg;
                StepConfig ci = s->cfg;  // stores and grouping as chosen; its own shape
                ci.threads = s->cfg_irr.threads;
                ci.wpe = s->cfg_irr.wpe;
                ci.regular = 0;
                e = launch_step(s->fp64, ai, ci, st);
            }
        } else {
            e = launch_step(s->fp64, a, s->cfg, st);
        }
        if (e != hipSuccess) return hip_fail(e, "step");
        if (s->korobov()) {
            KorArgs k{};
            k.f = a.f_out;
            k.table = s->kor();
            k.n_cells = s->n;
            k.p = int(s->kor_p);
            k.w0 = 8.0 * s->p.vmax[0] * s->p.vmax[0] * s->p.vmax[0] / double(s->kor_p);
            k.dt_kn = dt / s->p.tau_or_kn;
            k.vmax = s->p.vmax[0];
            k.g = s->g;
            k.flag = s->flag();
            e = launch_korobov(s->fp64, k, st);
            if (e != hipSuccess) return hip_fail(e, "Korobov collision");
        }
        s->cur ^= 1;
        s->steps++;
        if (s->p.check_every > 0 && s->steps % s->p.check_every == 0) {
            e = launch_global_sums(s->mom, s->tables, s->n, s->m->h0, s->partials(), kPartials, s->sums(), st);
            if (e != hipSuccess) return hip_fail(e, "global sums");
        }
    }
    return DVM_OK;
}

int dvm_global_sums(dvm_solver *s, void *stream) {
    clear_error();
    if (!s) return fail(DVM_ERR_ARG, "null solver");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    hipError_t e = launch_global_sums(s->mom, s->tables, s->n, s->m->h0, s->partials(), kPartials, s->sums(), S(stream));
    if (e != hipSuccess) return hip_fail(e, "global sums");
    return DVM_OK;
}

int dvm_current_f(const dvm_solver *s, void **f) {
    clear_error();
    if (!s || !f) return fail(DVM_ERR_ARG, "null argument");
    *f = s->f[s->cur];
    return DVM_OK;
}

int dvm_moments(dvm_solver *s, double *out, void *stream) {
    clear_error();
    if (!s || !out) return fail(DVM_ERR_ARG, "null argument");
    if (!s->f[0]) return fail(DVM_ERR_WORKSPACE, "solver not bound");
    if (s->hybrid_fluid && out == s->mom)
        return fail(DVM_ERR_ARG, "after hybrid steps the moments buffer holds the fluid cells' state: pass "
                                 "another output buffer");
    hipError_t e = launch_moments(s->fp64, s->f[s->cur], out, s->n, s->g, S(stream));
    // fluid cells of a hybrid step carry only their conserved moments
    if (e == hipSuccess) e = solver_fluid_moments(s, out, S(stream));
    if (e != hipSuccess) return hip_fail(e, "moments");
    return DVM_OK;
}

int dvm_check(dvm_solver *s, void *stream, dvm_diag *out) {
    clear_error();
    if (!s || !out) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    hipStream_t st = S(stream);
    hipError_t e = launch_global_sums(s->mom, s->tables, s->n, s->m->h0, s->partials(), kPartials, s->sums(), st);
    if (e != hipSuccess) return hip_fail(e, "global sums");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int flag = 0;
    e = hipMemcpy(out->sums, s->sums(), 5 * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&flag, s->flag(), sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(diag)");
    out->nonphysical = flag != 0;
    out->steps = s->steps;
    if (flag) return fail(DVM_ERR_NONPHYSICAL, "a cell reached rho <= 0, T <= 0 or NaN");
    return DVM_OK;
}

int dvm_f_to_canonical(const dvm_solver *s, const void *f_internal, void *f_canon, void *stream) {
    clear_error();
    if (!s || !f_internal || !f_canon) return fail(DVM_ERR_ARG, "null argument");
    hipError_t e = launch_to_canonical(s->fp64, true, f_internal, f_canon, s->n, s->nh, S(stream));
    if (e != hipSuccess) return hip_fail(e, "to_canonical");
    return DVM_OK;
}

int dvm_f_from_canonical(dvm_solver *s, const void *f_canon, void *f_internal, void *stream) {
    clear_error();
    if (!s || !f_internal || !f_canon) return fail(DVM_ERR_ARG, "null argument");
    hipError_t e = launch_to_canonical(s->fp64, false, f_canon, f_internal, s->n, s->nh, S(stream));
    if (e != hipSuccess) return hip_fail(e, "from_canonical");
    if (f_internal == s->f[s->cur] && s->uploaded) {
        // the buffer holds a new state: its moments, fresh hybrid masks
        e = launch_moments(s->fp64, f_internal, s->mom, s->n, s->g, S(stream));
        if (e != hipSuccess) return hip_fail(e, "moments");
        e = solver_reset_hybrid(s, S(stream));
        if (e != hipSuccess) return hip_fail(e, "hybrid masks");
        s->hybrid_fluid = false;
    }
    return DVM_OK;
}

int dvm_tune_shapes(const dvm_solver *s, int32_t *threads, int32_t *wpe, int32_t cap, int32_t *n) {
    clear_error();
    if (!s || !n || (cap > 0 && (!threads || !wpe))) return fail(DVM_ERR_ARG, "null argument");
    int t[64], w[64];
    const int total = list_kernels(s->nh, t, w, 64);
    for (int k = 0; k < total && k < cap && k < 64; ++k) {
        threads[k] = t[k];
        wpe[k] = w[k];
    }
    *n = total;
    return DVM_OK;
}

int dvm_tune_set(dvm_solver *s, int32_t threads, int32_t wpe, int32_t xcd_group, int32_t nt_store) {
    clear_error();
    if (!s) return fail(DVM_ERR_ARG, "null solver");
    if (xcd_group < 1 || xcd_group > 4096 || (xcd_group & (xcd_group - 1)))
        return fail(DVM_ERR_ARG, "xcd_group must be a power of two in [1, 4096]");
    if (!have_kernel(s->nh, threads, wpe))
        return fail(DVM_ERR_UNSUPPORTED, "no step kernel with %d threads, wpe %d for N = %d", threads, wpe, 2 * s->nh);
    s->cfg.threads = threads;
    s->cfg.wpe = wpe;
    s->cfg.xcd_group = xcd_group;
    s->cfg.nt_store = nt_store != 0;
    return DVM_OK;
}

int dvm_tune_get(const dvm_solver *s, int32_t *threads, int32_t *wpe, int32_t *xcd_group, int32_t *nt_store) {
    clear_error();
    if (!s || !threads || !wpe || !xcd_group || !nt_store) return fail(DVM_ERR_ARG, "null argument");
    *threads = s->cfg.threads;
    *wpe = s->cfg.wpe;
    *xcd_group = s->cfg.xcd_group;
    *nt_store = s->cfg.nt_store;
    return DVM_OK;
}

int dvm_tune_split(dvm_solver *s, int32_t enable, int32_t threads_irr, int32_t wpe_irr, int32_t *previous) {
    clear_error();
    if (!s) return fail(DVM_ERR_ARG, "null solver");
    if (previous) *previous = s->split ? 1 : 0;
    if (enable < 0) return DVM_OK;
    if (threads_irr > 0) {
        if (!have_kernel(s->nh, threads_irr, wpe_irr))
            return fail(DVM_ERR_UNSUPPORTED, "no step kernel with %d threads, wpe %d for N = %d", threads_irr, wpe_irr,
                        2 * s->nh);
        s->cfg_irr.threads = threads_irr;
        s->cfg_irr.wpe = wpe_irr;
    }
    s->split = enable != 0;
    return DVM_OK;
}

void dvm_destroy_solver(dvm_solver *s) { delete s; }

}  // extern "C"
