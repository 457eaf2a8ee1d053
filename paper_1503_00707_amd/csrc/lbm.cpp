// lbm.cpp -- host side of the lattice Boltzmann subset (section 4): the
// D3Q19 / D3Q27 solver object on a mesh, its compact cell records, buffer
// layout and launches on the caller's stream.  Like the DVM solver it holds no
// device memory of its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "solver_impl.h"

using namespace dvm;

struct dvm_lbm {
    const dvm_mesh *m = nullptr;
    dvm_lbm_params p{};
    bool fp64 = false;
    int64_t n = 0;
    size_t f_bytes = 0, mom_bytes = 0, tab_bytes = 0, ws_bytes = 0;
    size_t off_fine = 0;                 // fine list after the records in the tables buffer
    size_t off_part = 0, off_sums = 0, off_flag = 0;
    std::vector<LbmCell> cells;
    std::vector<int32_t> fine;
    void *f[2] = {nullptr, nullptr};
    int cur = 0;
    double *mom = nullptr;
    char *tables = nullptr, *ws = nullptr;
    bool uploaded = false;
    int64_t steps = 0;

    double *partials() const { return reinterpret_cast<double *>(ws + off_part); }
    double *sums() const { return reinterpret_cast<double *>(ws + off_sums); }
    int *flag() const { return reinterpret_cast<int *>(ws + off_flag); }
    const LbmCell *dcells() const { return reinterpret_cast<const LbmCell *>(tables); }
    const int32_t *dfine() const { return reinterpret_cast<const int32_t *>(tables + off_fine); }
};

namespace {
// the largest |c_x| + |c_y| + |c_z| of the lattice: 2 (D3Q19), 3 (D3Q27)
double max_speed_sum(int q) { return q == 19 ? 2.0 : 3.0; }
}  // namespace

extern "C" {

int dvm_lbm_create(const dvm_mesh *m, const dvm_lbm_params *p, dvm_lbm **out) {
    clear_error();
    if (!m || !p || !out) return fail(DVM_ERR_ARG, "null argument");
    *out = nullptr;
    if (p->q != 19 && p->q != 27) return fail(DVM_ERR_ARG, "q must be 19 or 27");
    if (p->precision != DVM_PREC_FP64 && p->precision != DVM_PREC_FP32) return fail(DVM_ERR_ARG, "bad precision");
    if (p->collision != DVM_COLL_EXP && p->collision != DVM_COLL_EULER)
        return fail(DVM_ERR_ARG, "collision must be DVM_COLL_EXP or DVM_COLL_EULER");
    if (!(p->tau > 0)) return fail(DVM_ERR_ARG, "tau must be > 0");
    if (m->device_tables) return fail(DVM_ERR_UNSUPPORTED, "the LBM path needs a mesh built by dvm_create_mesh");
    if (m->n_faces[DVM_FACE_INFLOW] || m->n_faces[DVM_FACE_WALL])
        return fail(DVM_ERR_UNSUPPORTED, "the LBM path has periodic and outflow boundaries only");
    dvm_lbm *s = new (std::nothrow) dvm_lbm();
    if (!s) return fail(DVM_ERR_ARG, "out of host memory");
    s->m = m;
    s->p = *p;
    s->fp64 = p->precision == DVM_PREC_FP64;
    s->n = int64_t(m->cells.size());
    s->cells.resize(size_t(s->n));
    for (int64_t c = 0; c < s->n; ++c) {
        const DevCell &d = m->table[size_t(c)];
        LbmCell &r = s->cells[size_t(c)];
        r.meta = uint32_t(d.level) << 24;
        r.fine = -1;
        for (int f = 0; f < 6; ++f) {
            r.meta |= uint32_t(d.type[f] & 7) << (3 * f);
            r.nb[f] = (d.type[f] == DVM_FACE_SAME || d.type[f] == DVM_FACE_COARSER) ? d.nbr[f][0] : -1;
            if (d.type[f] == DVM_FACE_FINER) {
                if (r.fine < 0) r.fine = int32_t(s->fine.size());
                for (int k = 0; k < 4; ++k) s->fine.push_back(d.nbr[f][k]);
            }
        }
    }
    const size_t fs = s->fp64 ? 8 : 4;
    s->f_bytes = align256(size_t(p->q) * size_t(s->n) * fs);
    s->mom_bytes = align256(size_t(5) * size_t(s->n) * 8);
    s->off_fine = align256(s->cells.size() * sizeof(LbmCell));
    s->tab_bytes = s->off_fine + align256(std::max<size_t>(s->fine.size(), 1) * 4);
    size_t o = 0;
    s->off_part = o; o += align256(size_t((s->n + 255) / 256) * 5 * 8);
    s->off_sums = o; o += 256;
    s->off_flag = o; o += 256;
    s->ws_bytes = o;
    *out = s;
    return DVM_OK;
}

int dvm_lbm_buffer_sizes(const dvm_lbm *s, dvm_sizes *out) {
    clear_error();
    if (!s || !out) return fail(DVM_ERR_ARG, "null argument");
    out->f_bytes = s->f_bytes;
    out->moments_bytes = s->mom_bytes;
    out->tables_bytes = s->tab_bytes;
    out->ws_bytes = s->ws_bytes;
    out->n_cells = s->n;
    out->nv_total = s->p.q;
    return DVM_OK;
}

int dvm_lbm_bind(dvm_lbm *s, void *f_a, void *f_b, double *moments, void *tables, void *ws) {
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
    s->tables = static_cast<char *>(tables);
    s->ws = static_cast<char *>(ws);
    s->uploaded = false;
    s->steps = 0;
    return DVM_OK;
}

int dvm_lbm_upload(dvm_lbm *s, void *stream) {
    clear_error();
    if (!s || !s->ws) return fail(DVM_ERR_WORKSPACE, "solver not bound");
    hipStream_t st = S(stream);
    hipError_t e = hipMemcpyAsync(s->tables, s->cells.data(), s->cells.size() * sizeof(LbmCell),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !s->fine.empty())
        e = hipMemcpyAsync(s->tables + s->off_fine, s->fine.data(), s->fine.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(s->ws, 0, s->ws_bytes, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host tables stay valid until copied
    if (e != hipSuccess) return hip_fail(e, "LBM upload");
    s->uploaded = true;
    return DVM_OK;
}

int dvm_lbm_init(dvm_lbm *s, const double *prim, void *stream) {
    clear_error();
    if (!s || !prim) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_lbm_upload first");
    s->cur = 0;
    s->steps = 0;
    hipError_t e = launch_lbm_init(s->p.q, s->fp64, prim, s->f[0], s->n, s->flag(), S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "LBM init");
}

int dvm_lbm_dt(const dvm_lbm *s, double cfl, double *dt) {
    clear_error();
    if (!s || !dt) return fail(DVM_ERR_ARG, "null argument");
    if (!(cfl > 0)) return fail(DVM_ERR_ARG, "cfl must be > 0");
    *dt = cfl * s->m->h_min / max_speed_sum(s->p.q);
    return DVM_OK;
}

int dvm_lbm_step(dvm_lbm *s, int32_t n_steps, double dt, double cfl, void *stream) {
    clear_error();
    if (!s) return fail(DVM_ERR_ARG, "null solver");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_lbm_upload first");
    if (n_steps < 0) return fail(DVM_ERR_ARG, "n_steps < 0");
    if (!(dt > 0)) {
        int rc = dvm_lbm_dt(s, cfl, &dt);
        if (rc) return rc;
    }
    LbmArgs a{};
    a.cells = s->dcells();
    a.fine = s->dfine();
    a.n = s->n;
    a.dt = dt;
    a.h0 = s->m->h0;
    a.euler = s->p.collision == DVM_COLL_EULER;
    a.relax = a.euler ? dt / s->p.tau : std::exp(-dt / s->p.tau);
    a.xcd_log2 = 5;  // 8,192 consecutive cells per XCD run: their face neighbours share that XCD's L2
    a.flag = s->flag();
    for (int it = 0; it < n_steps; ++it) {
        a.f_in = s->f[s->cur];
        a.f_out = s->f[s->cur ^ 1];
        hipError_t e = launch_lbm_step(s->p.q, s->fp64, a, S(stream));
        if (e != hipSuccess) return hip_fail(e, "LBM step");
        s->cur ^= 1;
        s->steps++;
    }
    return DVM_OK;
}

int dvm_lbm_moments(dvm_lbm *s, double *out, void *stream) {
    clear_error();
    if (!s || !out) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_lbm_upload first");
    hipError_t e = launch_lbm_moments(s->p.q, s->fp64, s->f[s->cur], s->dcells(), s->n, s->m->h0, out,
                                      s->partials(), nullptr, S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "LBM moments");
}

int dvm_lbm_check(dvm_lbm *s, void *stream, dvm_diag *out) {
    clear_error();
    if (!s || !out) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_lbm_upload first");
    hipStream_t st = S(stream);
    hipError_t e = launch_lbm_moments(s->p.q, s->fp64, s->f[s->cur], s->dcells(), s->n, s->m->h0, s->mom,
                                      s->partials(), s->sums(), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpy(out->sums, s->sums(), 5 * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&flag, s->flag(), sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "LBM check");
    out->nonphysical = flag != 0;
    out->steps = s->steps;
    if (flag) return fail(DVM_ERR_NONPHYSICAL, "a cell reached rho <= 0 or NaN");
    return DVM_OK;
}

int dvm_lbm_get_f(const dvm_lbm *s, void *out, void *stream) {
    clear_error();
    if (!s || !out) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_lbm_upload first");
    hipError_t e = launch_lbm_canon(s->p.q, s->fp64, s->f[s->cur], out, s->n, true, S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "LBM f");
}

int dvm_lbm_set_f(dvm_lbm *s, const void *in, void *stream) {
    clear_error();
    if (!s || !in) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_lbm_upload first");
    hipError_t e = launch_lbm_canon(s->p.q, s->fp64, in, s->f[s->cur], s->n, false, S(stream));
    return e == hipSuccess ? DVM_OK : hip_fail(e, "LBM f");
}

int dvm_lbm_current_f(const dvm_lbm *s, void **f) {
    clear_error();
    if (!s || !f) return fail(DVM_ERR_ARG, "null argument");
    *f = s->f[s->cur];
    return DVM_OK;
}

void dvm_destroy_lbm(dvm_lbm *s) { delete s; }

}  // extern "C"
