// batch.cpp -- many independent solvers advanced together: per velocity-grid
// size one batched step kernel over the cells of all its instances, then one
// batched global-sum pair, recorded once into a HIP graph per buffer parity
// and replayed with a single graph launch per step.  A project-written
// autotuner times the compiled kernel shapes on the batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "solver_impl.h"

using namespace dvm;

namespace {

struct Group {
    int nh = 0;
    std::vector<int> inst;         // instance indices, decreasing cost
    std::vector<uint32_t> wg_end;  // cumulative cells (one workgroup per cell)
    StepConfig cfg{};
    size_t off_args[2] = {0, 0};   // StepArgs[n] for each buffer parity
    size_t off_end = 0;            // uint32_t[n]
    double tuned_ms = 0.0;
};

}  // namespace

struct dvm_batch {
    std::vector<dvm_solver *> s;
    std::vector<double> dt;
    std::vector<int> base_cur;     // s[i]->cur when the arguments were written
    bool fp64 = false;
    std::vector<Group> groups;
    size_t off_sums[2] = {0, 0};   // SumArgs[n] (identical for both parities)
    size_t ws_bytes = 0;
    char *ws = nullptr;
    bool args_valid = false;
    bool branches = true;          // groups on parallel graph branches (else one chain)
    int phase = 0;                 // buffer parity of the next step
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    // host copy of the argument block (kept alive for the asynchronous upload)
    std::vector<char> host;

    void drop_graphs() {
        for (auto &g : graph)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    ~dvm_batch() { drop_graphs(); }
};

namespace {

// Write the argument block for the current buffers of every instance.
int write_args(dvm_batch *b, hipStream_t st) {
    b->host.assign(b->ws_bytes, 0);
    for (size_t i = 0; i < b->s.size(); ++i) b->base_cur[i] = b->s[i]->cur;
    for (auto &g : b->groups) {
        for (int ph = 0; ph < 2; ++ph) {
            StepArgs *args = reinterpret_cast<StepArgs *>(b->host.data() + g.off_args[ph]);
            for (size_t k = 0; k < g.inst.size(); ++k) {
                const int i = g.inst[k];
                const dvm_solver *s = b->s[i];
                StepArgs a = solver_step_args(s, b->dt[i]);
                a.f_in = s->f[s->cur ^ ph];
                a.f_out = s->f[s->cur ^ ph ^ 1];
                args[k] = a;
            }
        }
        std::memcpy(b->host.data() + g.off_end, g.wg_end.data(), g.wg_end.size() * sizeof(uint32_t));
    }
    SumArgs *sa = reinterpret_cast<SumArgs *>(b->host.data() + b->off_sums[0]);
    for (size_t i = 0; i < b->s.size(); ++i) {
        const dvm_solver *s = b->s[i];
        sa[i] = SumArgs{s->mom, s->tables, s->n, s->m->h0, s->partials(), s->sums()};
    }
    hipError_t e = hipMemcpyAsync(b->ws, b->host.data(), b->ws_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch arguments)");
    e = hipStreamSynchronize(st);  // the host block may be rewritten by the next call
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    b->args_valid = true;
    b->phase = 0;
    return DVM_OK;
}

hipError_t enqueue_group(const dvm_batch *b, const Group &g, int ph, const StepConfig &cfg, hipStream_t st) {
    return launch_step_batch(b->fp64, reinterpret_cast<const StepArgs *>(b->ws + g.off_args[ph]),
                             reinterpret_cast<const uint32_t *>(b->ws + g.off_end), int(g.inst.size()),
                             g.wg_end.back(), g.nh, cfg, st);
}

hipError_t enqueue_step(const dvm_batch *b, int ph, hipStream_t st) {
    for (const auto &g : b->groups) {
        hipError_t e = enqueue_group(b, g, ph, g.cfg, st);
        if (e != hipSuccess) return e;
    }
    return launch_global_sums_batch(reinterpret_cast<const SumArgs *>(b->ws + b->off_sums[0]), int(b->s.size()),
                                    kPartials, st);
}

// The step with the velocity-grid groups on parallel branches: group k > 0 is
// enqueued on side stream k - 1, forked from and joined back into st by
// events, so that in the recorded graph the groups' kernels are independent
// nodes (the instances of different groups share no data) and run
// concurrently; the global sums follow the join.
hipError_t enqueue_step_branches(const dvm_batch *b, int ph, hipStream_t st, const std::vector<hipStream_t> &side,
                                 const std::vector<hipEvent_t> &ev) {
    hipError_t e = hipEventRecord(ev[0], st);
    for (size_t k = 1; k < b->groups.size() && e == hipSuccess; ++k) e = hipStreamWaitEvent(side[k - 1], ev[0], 0);
    for (size_t k = 0; k < b->groups.size() && e == hipSuccess; ++k)
        e = enqueue_group(b, b->groups[k], ph, b->groups[k].cfg, k == 0 ? st : side[k - 1]);
    for (size_t k = 1; k < b->groups.size() && e == hipSuccess; ++k) {
        e = hipEventRecord(ev[k], side[k - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev[k], 0);
    }
    if (e != hipSuccess) return e;
    return launch_global_sums_batch(reinterpret_cast<const SumArgs *>(b->ws + b->off_sums[0]), int(b->s.size()),
                                    kPartials, st);
}

int build_graphs(dvm_batch *b) {
    hipStream_t cap;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    // side streams and events of the parallel branches (default priority)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;
    int rc = DVM_OK;
    for (size_t k = 1; k < b->groups.size() && rc == DVM_OK; ++k) {
        hipStream_t x;
        e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamCreate");
        else side.push_back(x);
    }
    for (size_t k = 0; k < b->groups.size() && rc == DVM_OK; ++k) {
        hipEvent_t x;
        e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
        if (e != hipSuccess) rc = hip_fail(e, "hipEventCreate");
        else ev.push_back(x);
    }
    for (int ph = 0; ph < 2 && rc == DVM_OK; ++ph) {
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            rc = hip_fail(e, "hipStreamBeginCapture");
            break;
        }
        hipError_t el = b->branches ? enqueue_step_branches(b, ph, cap, side, ev) : enqueue_step(b, ph, cap);
        e = hipStreamEndCapture(cap, &graph);
        if (el != hipSuccess) rc = hip_fail(el, "batched step (capture)");
        else if (e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
        else {
            e = hipGraphInstantiate(&b->graph[ph], graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
        }
        if (graph) (void)hipGraphDestroy(graph);
    }
    (void)hipStreamDestroy(cap);
    for (auto x : side) (void)hipStreamDestroy(x);
    for (auto x : ev) (void)hipEventDestroy(x);
    if (rc != DVM_OK) b->drop_graphs();
    return rc;
}

// Instances stepped on their own since the arguments were written: rewrite.
bool in_step(const dvm_batch *b) {
    for (size_t i = 0; i < b->s.size(); ++i)
        if (b->s[i]->cur != (b->base_cur[i] ^ b->phase)) return false;
    return true;
}

}  // namespace

extern "C" {

int dvm_batch_create(dvm_solver *const *solvers, int32_t n, double cfl, dvm_batch **out) {
    clear_error();
    if (!solvers || !out || n <= 0) return fail(DVM_ERR_ARG, "need n > 0 solvers");
    if (!(cfl > 0)) return fail(DVM_ERR_ARG, "cfl must be > 0");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        const dvm_solver *s = solvers[i];
        if (!s) return fail(DVM_ERR_ARG, "solver %d is NULL", i);
        if (s->fp64 != solvers[0]->fp64) return fail(DVM_ERR_UNSUPPORTED, "a batch has one storage precision");
        if (s->muscl) return fail(DVM_ERR_UNSUPPORTED, "batched steps are first order");
        if (s->korobov()) return fail(DVM_ERR_UNSUPPORTED, "batched steps relax with BGK");
        if (s->hybrid_fluid)
            return fail(DVM_ERR_UNSUPPORTED, "solver %d holds fluid cells from hybrid steps (their f is stale)", i);
        if (uint64_t(s->n) >= (uint64_t(1) << 31)) return fail(DVM_ERR_UNSUPPORTED, "instance too large");
        for (int j = 0; j < i; ++j)
            if (solvers[j] == s) return fail(DVM_ERR_ARG, "solver %d listed twice", i);
    }
    dvm_batch *b = new (std::nothrow) dvm_batch();
    if (!b) return fail(DVM_ERR_ARG, "out of host memory");
    b->s.assign(solvers, solvers + n);
    b->fp64 = solvers[0]->fp64;
    b->base_cur.assign(n, 0);
    for (int i = 0; i < n; ++i) b->dt.push_back(cfl * solvers[i]->m->h_min / solver_max_speed_sum(solvers[i]));
    // groups by velocity grid, instances by decreasing cost (cells x velocities)
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return double(solvers[x]->n) * double(solvers[x]->nv) > double(solvers[y]->n) * double(solvers[y]->nv);
    });
    for (int i : order) {
        auto it = std::find_if(b->groups.begin(), b->groups.end(), [&](const Group &g) { return g.nh == solvers[i]->nh; });
        if (it == b->groups.end()) {
            b->groups.push_back(Group{});
            it = b->groups.end() - 1;
            it->nh = solvers[i]->nh;
            it->cfg = solvers[i]->cfg;
        }
        it->inst.push_back(i);
        const uint64_t prev = it->wg_end.empty() ? 0 : it->wg_end.back();
        if (prev + uint64_t(solvers[i]->n) >= (uint64_t(1) << 31)) {
            delete b;
            return fail(DVM_ERR_UNSUPPORTED, "more than 2^31 cells share one velocity grid");
        }
        it->wg_end.push_back(uint32_t(prev + solvers[i]->n));
    }
    std::sort(b->groups.begin(), b->groups.end(), [](const Group &x, const Group &y) { return x.nh > y.nh; });
    size_t o = 0;
    for (auto &g : b->groups) {
        for (int ph = 0; ph < 2; ++ph) {
            g.off_args[ph] = o;
            o += align256(g.inst.size() * sizeof(StepArgs));
        }
        g.off_end = o;
        o += align256(g.inst.size() * sizeof(uint32_t));
    }
    b->off_sums[0] = b->off_sums[1] = o;
    o += align256(size_t(n) * sizeof(SumArgs));
    b->ws_bytes = o;
    *out = b;
    return DVM_OK;
}

int dvm_batch_workspace_bytes(const dvm_batch *b, size_t *bytes) {
    clear_error();
    if (!b || !bytes) return fail(DVM_ERR_ARG, "null argument");
    *bytes = b->ws_bytes;
    return DVM_OK;
}

int dvm_batch_bind(dvm_batch *b, void *ws) {
    clear_error();
    if (!b || !ws) return fail(DVM_ERR_ARG, "null argument");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(DVM_ERR_ARG, "workspace must be 256-byte aligned");
    b->ws = static_cast<char *>(ws);
    b->args_valid = false;
    b->drop_graphs();
    return DVM_OK;
}

int dvm_batch_step(dvm_batch *b, int32_t n_steps, void *stream) {
    clear_error();
    if (!b) return fail(DVM_ERR_ARG, "null batch");
    if (!b->ws) return fail(DVM_ERR_WORKSPACE, "call dvm_batch_bind first");
    if (n_steps < 0) return fail(DVM_ERR_ARG, "n_steps < 0");
    hipStream_t st = S(stream);
    for (auto *s : b->s) {
        if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "every solver must be bound and uploaded");
        if (s->hybrid_fluid)
            return fail(DVM_ERR_UNSUPPORTED, "a solver holds fluid cells from hybrid steps (their f is stale)");
    }
    if (!b->args_valid || !in_step(b)) {
        // the graphs read the argument block by address: no re-capture needed
        int rc = write_args(b, st);
        if (rc) return rc;
    }
    if (!b->graph[0]) {
        int rc = build_graphs(b);
        if (rc) return rc;
    }
    for (int it = 0; it < n_steps; ++it) {
        hipError_t e = hipGraphLaunch(b->graph[b->phase], st);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        b->phase ^= 1;
        for (auto *s : b->s) {
            s->cur ^= 1;
            s->steps++;
        }
    }
    return DVM_OK;
}

int dvm_batch_tune(dvm_batch *b, int32_t reps, const char *cache_path, void *stream) {
    clear_error();
    if (!b) return fail(DVM_ERR_ARG, "null batch");
    if (!b->ws) return fail(DVM_ERR_WORKSPACE, "call dvm_batch_bind first");
    if (reps < 1) return fail(DVM_ERR_ARG, "reps must be >= 1");
    hipStream_t st = S(stream);
    for (auto *s : b->s) {
        if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "every solver must be bound and uploaded");
        if (s->hybrid_fluid)
            return fail(DVM_ERR_UNSUPPORTED, "a solver holds fluid cells from hybrid steps (their f is stale)");
    }
    if (!b->args_valid || !in_step(b)) {
        int rc = write_args(b, st);
        if (rc) return rc;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(DVM_ERR_DEVICE, "events");
    const int groups[3] = {1, 8, 64};
    int rc = DVM_OK;
    bool timed = false;
    for (auto &g : b->groups) {
        const TuneKey key{"batch", g.nh, b->fp64 ? 1 : 0, 0};
        StepConfig cached{};
        double cached_ms = 0.0;
        if (tune_cache_get(cache_path, key, &cached, &cached_ms) && have_kernel(g.nh, cached.threads, cached.wpe) &&
            cached.xcd_group >= 1 && cached.xcd_group <= 4096 && !(cached.xcd_group & (cached.xcd_group - 1))) {
            g.cfg = StepConfig{cached.threads, cached.xcd_group, cached.nt_store != 0, cached.wpe, 0};
            g.tuned_ms = cached_ms;
            continue;
        }
        timed = true;
        // trial steps read the current buffers and write only the next ones
        // (and the moments), so the state the batch advances is unchanged
        int thr[64], wpe[64];
        const int nk = std::min(list_kernels(g.nh, thr, wpe, 64), 64);
        double best = 1e300;
        StepConfig best_cfg = g.cfg;
        for (int k = 0; k < nk && rc == DVM_OK; ++k)
            for (int xg : groups)
                for (int nt = 0; nt < 2 && rc == DVM_OK; ++nt) {
                    const StepConfig c{thr[k], xg, nt, wpe[k]};
                    hipError_t e = enqueue_group(b, g, b->phase, c, st);  // warm-up
                    if (e == hipSuccess) e = hipEventRecord(e0, st);
                    for (int r = 0; r < reps && e == hipSuccess; ++r) e = enqueue_group(b, g, b->phase, c, st);
                    if (e == hipSuccess) e = hipEventRecord(e1, st);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e != hipSuccess) {
                        rc = hip_fail(e, "tuning launch");
                        break;
                    }
                    if (ms / reps < best) {
                        best = ms / reps;
                        best_cfg = c;
                    }
                }
        g.cfg = best_cfg;
        g.tuned_ms = best;
        if (rc == DVM_OK) rc = tune_cache_put(cache_path, key, best_cfg, best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    b->drop_graphs();  // new kernel shapes: re-record at the next step
    if (!timed) return DVM_OK;
    // the trial steps overwrote the moments: restore those of the current state
    for (auto *s : b->s) {
        hipError_t e = launch_moments(s->fp64, s->f[s->cur], s->mom, s->n, s->g, st);
        if (e != hipSuccess) return hip_fail(e, "moments");
    }
    return DVM_OK;
}

int dvm_batch_branches(dvm_batch *b, int32_t enable, int32_t *previous) {
    clear_error();
    if (!b) return fail(DVM_ERR_ARG, "null batch");
    if (previous) *previous = b->branches ? 1 : 0;
    if (enable < 0) return DVM_OK;
    if ((enable != 0) != b->branches) {
        b->branches = enable != 0;
        b->drop_graphs();  // re-record at the next step
    }
    return DVM_OK;
}

int dvm_batch_info(const dvm_batch *b, int32_t group, int32_t *nh, int32_t *n_inst, int64_t *n_cells,
                   int32_t *threads, int32_t *wpe, int32_t *xcd_group, int32_t *nt_store, double *tuned_ms) {
    clear_error();
    if (!b) return fail(DVM_ERR_ARG, "null batch");
    if (group < 0) {
        if (n_inst) *n_inst = int32_t(b->groups.size());
        return DVM_OK;
    }
    if (group >= int32_t(b->groups.size())) return fail(DVM_ERR_ARG, "no group %d", group);
    const Group &g = b->groups[group];
    if (nh) *nh = g.nh;
    if (n_inst) *n_inst = int32_t(g.inst.size());
    if (n_cells) *n_cells = g.wg_end.back();
    if (threads) *threads = g.cfg.threads;
    if (wpe) *wpe = g.cfg.wpe;
    if (xcd_group) *xcd_group = g.cfg.xcd_group;
    if (nt_store) *nt_store = g.cfg.nt_store;
    if (tuned_ms) *tuned_ms = g.tuned_ms;
    return DVM_OK;
}

void dvm_destroy_batch(dvm_batch *b) { delete b; }

}  // extern "C"
