// persist.cpp -- what outlives a process: the solver's state in a checkpoint
// file (dvm_save / dvm_load) and the autotuner's choices in a cache file
// keyed by GPU architecture, velocity grid, precision and scheme (dvm_tune,
// dvm_batch_tune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "solver_impl.h"

using namespace dvm;

namespace {

// ---- checkpoint file ------------------------------------------------------

constexpr char kMagic[8] = {'D', 'V', 'M', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t kVersion = 1;

struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t nh;
    int64_t n_cells;
    int32_t precision;
    int32_t scheme;
    int64_t steps;
    double vmax[3];
    int32_t base[3];
    int32_t bc[6];
    double h0;
    int32_t hybrid;        // the file holds the hybrid step's previous mask
    int32_t hybrid_fluid;  // fluid cells hold only their moments
    int32_t has_net;       // the file holds a network (parameters, Adam state)
    int32_t pad;
    int64_t net_t;         // Adam step count
};

// FNV-1a, 64 bit, over every byte after the header's checksum field
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    }
};

struct File {
    FILE *fp = nullptr;
    Fnv sum;
    ~File() {
        if (fp) std::fclose(fp);
    }
    bool write(const void *p, size_t n) {
        sum.add(p, n);
        return std::fwrite(p, 1, n, fp) == n;
    }
    bool read(void *p, size_t n) {
        if (std::fread(p, 1, n, fp) != n) return false;
        sum.add(p, n);
        return true;
    }
};

constexpr size_t kChunk = size_t(64) << 20;  // host staging for device <-> file copies

// device [bytes] -> file, through a host chunk
int dev_to_file(File &f, const void *dev, size_t bytes, hipStream_t st) {
    std::vector<char> buf(std::min(bytes, kChunk));
    for (size_t o = 0; o < bytes; o += kChunk) {
        const size_t n = std::min(kChunk, bytes - o);
        hipError_t e = hipMemcpyAsync(buf.data(), static_cast<const char *>(dev) + o, n, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(checkpoint)");
        if (!f.write(buf.data(), n)) return fail(DVM_ERR_ARG, "checkpoint write failed: %s", std::strerror(errno));
    }
    return DVM_OK;
}

int file_to_dev(File &f, void *dev, size_t bytes, hipStream_t st) {
    std::vector<char> buf(std::min(bytes, kChunk));
    for (size_t o = 0; o < bytes; o += kChunk) {
        const size_t n = std::min(kChunk, bytes - o);
        if (!f.read(buf.data(), n)) return fail(DVM_ERR_ARG, "checkpoint file is truncated");
        hipError_t e = hipMemcpyAsync(static_cast<char *>(dev) + o, buf.data(), n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(checkpoint)");
    }
    return DVM_OK;
}

// ---- tuner cache ----------------------------------------------------------

std::string key_text(const TuneKey &k, const std::string &arch) {
    std::ostringstream o;
    o << k.kind << ' ' << arch << " nh=" << k.nh << " fp64=" << k.fp64 << " scheme=" << k.scheme;
    return o.str();
}

// the solver's trial step: reads f[cur], writes f[cur ^ 1] and the moments;
// the state it advances is unchanged
hipError_t trial_step(const dvm_solver *s, const StepConfig &cfg, double dt, hipStream_t st) {
    StepArgs a = solver_step_args(s, dt);
    a.xcd_log2 = 0;
    while ((1 << (a.xcd_log2 + 1)) <= cfg.xcd_group) ++a.xcd_log2;
    a.f_in = s->f[s->cur];
    a.f_out = s->f[s->cur ^ 1];
    return launch_step(s->fp64, a, cfg, st);
}

}  // namespace

namespace dvm {

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "";
    std::string a = p.gcnArchName;
    const size_t colon = a.find(':');  // drop feature suffixes (":sramecc+:xnack-")
    return colon == std::string::npos ? a : a.substr(0, colon);
}

bool tune_cache_get(const char *path, const TuneKey &k, StepConfig *cfg, double *ms) {
    return tune_cache_get_arch(path, k, device_arch(), cfg, ms);
}

int tune_cache_put(const char *path, const TuneKey &k, const StepConfig &cfg, double ms) {
    return tune_cache_put_arch(path, k, device_arch(), cfg, ms);
}

bool tune_cache_get_arch(const char *path, const TuneKey &k, const std::string &arch, StepConfig *cfg, double *ms) {
    if (!path) return false;
    std::ifstream in(path);
    if (!in) return false;
    const std::string want = key_text(k, arch);
    std::string line;
    while (std::getline(in, line)) {
        const size_t bar = line.find(" | ");
        if (bar == std::string::npos || line.compare(0, bar, want) != 0 || bar != want.size()) continue;
        StepConfig c{};
        double t = 0.0;
        if (std::sscanf(line.c_str() + bar + 3, "threads=%d wpe=%d xcd_group=%d nt_store=%d ms=%lf", &c.threads, &c.wpe,
                        &c.xcd_group, &c.nt_store, &t) != 5)
            continue;
        *cfg = c;
        if (ms) *ms = t;
        return true;
    }
    return false;
}

int tune_cache_put_arch(const char *path, const TuneKey &k, const std::string &arch, const StepConfig &cfg,
                        double ms) {
    if (!path) return DVM_OK;
    if (arch.empty() || arch.find_first_of(" |\n") != std::string::npos)
        return fail(DVM_ERR_ARG, "bad architecture name for the tuner cache");
    const std::string key = key_text(k, arch);
    std::vector<std::string> lines;
    {
        std::ifstream in(path);
        std::string line;
        while (in && std::getline(in, line))
            if (line.compare(0, key.size() + 3, key + " | ") != 0) lines.push_back(line);
    }
    char val[160];
    std::snprintf(val, sizeof val, "threads=%d wpe=%d xcd_group=%d nt_store=%d ms=%.6f", cfg.threads, cfg.wpe,
                  cfg.xcd_group, cfg.nt_store, ms);
    lines.push_back(key + " | " + val);
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out) return fail(DVM_ERR_ARG, "cannot write the tuner cache %s", tmp.c_str());
        for (auto &l : lines) out << l << '\n';
        if (!out) return fail(DVM_ERR_ARG, "cannot write the tuner cache %s", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0) return fail(DVM_ERR_ARG, "cannot replace the tuner cache %s", path);
    return DVM_OK;
}

}  // namespace dvm

extern "C" {

int dvm_tune_cache_get(const char *path, const char *kind, const char *arch, int32_t nh, int32_t fp64,
                       int32_t scheme, int32_t shape[4], double *ms, int32_t *found) {
    clear_error();
    if (!path || !kind || !arch || !shape || !found) return fail(DVM_ERR_ARG, "null argument");
    StepConfig c{};
    double t = 0.0;
    *found = tune_cache_get_arch(path, TuneKey{kind, nh, fp64 ? 1 : 0, scheme}, arch, &c, &t) ? 1 : 0;
    if (*found) {
        shape[0] = c.threads;
        shape[1] = c.wpe;
        shape[2] = c.xcd_group;
        shape[3] = c.nt_store;
        if (ms) *ms = t;
    }
    return DVM_OK;
}

int dvm_tune_cache_put(const char *path, const char *kind, const char *arch, int32_t nh, int32_t fp64,
                       int32_t scheme, const int32_t shape[4], double ms) {
    clear_error();
    if (!path || !kind || !arch || !shape) return fail(DVM_ERR_ARG, "null argument");
    if (std::strcmp(kind, "step") != 0 && std::strcmp(kind, "batch") != 0)
        return fail(DVM_ERR_ARG, "kind must be \"step\" or \"batch\"");
    const StepConfig c{shape[0], shape[2], shape[3], shape[1], 0};
    return tune_cache_put_arch(path, TuneKey{kind, nh, fp64 ? 1 : 0, scheme}, arch, c, ms);
}

int dvm_tune(dvm_solver *s, const char *cache_path, int32_t reps, int32_t *from_cache, void *stream) {
    clear_error();
    if (!s) return fail(DVM_ERR_ARG, "null solver");
    if (from_cache) *from_cache = 0;
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    if (s->hybrid_fluid) return fail(DVM_ERR_UNSUPPORTED, "fluid cells hold no f: tune before hybrid steps");
    if (reps < 1) return fail(DVM_ERR_ARG, "reps must be >= 1");
    const TuneKey key{"step", s->nh, s->fp64 ? 1 : 0, s->muscl ? 1 : 0};
    StepConfig c{};
    if (tune_cache_get(cache_path, key, &c, nullptr) && have_kernel(s->nh, c.threads, c.wpe) && c.xcd_group >= 1 &&
        c.xcd_group <= 4096 && !(c.xcd_group & (c.xcd_group - 1))) {
        s->cfg.threads = c.threads;
        s->cfg.wpe = c.wpe;
        s->cfg.xcd_group = c.xcd_group;
        s->cfg.nt_store = c.nt_store != 0;
        if (from_cache) *from_cache = 1;
        return DVM_OK;
    }
    hipStream_t st = S(stream);
    hipError_t e = hipSuccess;
    double dt = 0.0;
    int rc = dvm_dt(s, 0.5, &dt);
    if (rc) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(DVM_ERR_DEVICE, "events");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(DVM_ERR_DEVICE, "events");
    }
    int thr[64], wpe[64];
    const int nk = std::min(list_kernels(s->nh, thr, wpe, 64), 64);
    const int groups[4] = {1, 8, 64, 512};
    double best = 1e300;
    StepConfig best_cfg = s->cfg;
    for (int k = 0; k < nk && rc == DVM_OK; ++k)
        for (int xg : groups)
            for (int nt = 0; nt < 2 && rc == DVM_OK; ++nt) {
                const StepConfig cfg{thr[k], xg, nt, wpe[k], 0};
                e = trial_step(s, cfg, dt, st);  // warm-up
                if (e == hipSuccess) e = hipEventRecord(e0, st);
                for (int r = 0; r < reps && e == hipSuccess; ++r) e = trial_step(s, cfg, dt, st);
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
                    best_cfg = cfg;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    // the trial steps overwrote the moments buffer: those of the current state
    e = launch_moments(s->fp64, s->f[s->cur], s->mom, s->n, s->g, st);
    if (e != hipSuccess) return hip_fail(e, "moments");
    s->cfg.threads = best_cfg.threads;
    s->cfg.wpe = best_cfg.wpe;
    s->cfg.xcd_group = best_cfg.xcd_group;
    s->cfg.nt_store = best_cfg.nt_store;
    return tune_cache_put(cache_path, key, best_cfg, best);
}

int dvm_save(dvm_solver *s, const dvm_mlp *net, const char *path, void *stream) {
    clear_error();
    if (!s || !path) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    if (net && (!net->params || !net->ws)) return fail(DVM_ERR_WORKSPACE, "network not bound");
    hipStream_t st = S(stream);
    // canonical velocity order, staged in the other state buffer (the next
    // step overwrites it anyway)
    void *stage = s->f[s->cur ^ 1];
    int rc = dvm_f_to_canonical(s, s->f[s->cur], stage, stream);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    File f;
    const std::string tmp = std::string(path) + ".tmp";
    f.fp = std::fopen(tmp.c_str(), "wb");
    if (!f.fp) return fail(DVM_ERR_ARG, "cannot open %s: %s", tmp.c_str(), std::strerror(errno));
    CkptHeader h{};
    std::memcpy(h.magic, kMagic, 8);
    h.version = kVersion;
    h.nh = s->nh;
    h.n_cells = s->n;
    h.precision = s->p.precision;
    h.scheme = s->p.scheme;
    h.steps = s->steps;
    for (int b = 0; b < 3; ++b) h.vmax[b] = s->p.vmax[b];
    for (int b = 0; b < 3; ++b) h.base[b] = s->m->base[b];
    for (int b = 0; b < 6; ++b) h.bc[b] = s->m->bc[b];
    h.h0 = s->m->h0;
    h.hybrid = s->hybrid ? 1 : 0;
    h.hybrid_fluid = s->hybrid_fluid ? 1 : 0;
    h.has_net = net ? 1 : 0;
    h.net_t = net ? net->t : 0;
    bool ok = f.write(&h, sizeof h);
    // the leaf list in cell (Morton) order
    for (const Leaf &l : s->m->cells) {
        const int32_t ijk[3] = {l.i, l.j, l.k};
        ok = ok && f.write(&l.key, 8) && f.write(&l.level, 1) && f.write(ijk, 12);
    }
    if (!ok) return fail(DVM_ERR_ARG, "checkpoint write failed: %s", std::strerror(errno));
    rc = dev_to_file(f, stage, size_t(s->n) * size_t(s->nv) * (s->fp64 ? 8 : 4), st);
    if (!rc) rc = dev_to_file(f, s->mom, size_t(5) * size_t(s->n) * 8, st);
    if (!rc && s->hybrid) rc = dev_to_file(f, solver_hybrid_prev(s), size_t(s->n), st);
    if (!rc && net) {
        rc = dev_to_file(f, net->params, size_t(kMlpParams) * 4, st);
        if (!rc) rc = dev_to_file(f, net->m(), size_t(kMlpWeights) * 4, st);
        if (!rc) rc = dev_to_file(f, net->v(), size_t(kMlpWeights) * 4, st);
    }
    if (rc) return rc;
    const uint64_t sum = f.sum.h;
    if (std::fwrite(&sum, 1, 8, f.fp) != 8 || std::fclose(f.fp) != 0) {
        f.fp = nullptr;
        return fail(DVM_ERR_ARG, "checkpoint write failed: %s", std::strerror(errno));
    }
    f.fp = nullptr;
    if (std::rename(tmp.c_str(), path) != 0) return fail(DVM_ERR_ARG, "cannot rename %s", tmp.c_str());
    return DVM_OK;
}

int dvm_load(dvm_solver *s, dvm_mlp *net, const char *path, void *stream) {
    clear_error();
    if (!s || !path) return fail(DVM_ERR_ARG, "null argument");
    if (!s->uploaded) return fail(DVM_ERR_WORKSPACE, "call dvm_upload first");
    if (net && (!net->params || !net->ws)) return fail(DVM_ERR_WORKSPACE, "network not bound");
    hipStream_t st = S(stream);
    File f;
    f.fp = std::fopen(path, "rb");
    if (!f.fp) return fail(DVM_ERR_ARG, "cannot open %s: %s", path, std::strerror(errno));
    CkptHeader h{};
    if (!f.read(&h, sizeof h) || std::memcmp(h.magic, kMagic, 8) != 0 || h.version != kVersion)
        return fail(DVM_ERR_ARG, "%s is not a checkpoint of this library", path);
    bool same = h.nh == s->nh && h.n_cells == s->n && h.precision == s->p.precision && h.scheme == s->p.scheme &&
                h.h0 == s->m->h0;
    for (int b = 0; b < 3; ++b) same = same && h.vmax[b] == s->p.vmax[b] && h.base[b] == s->m->base[b];
    for (int b = 0; b < 6; ++b) same = same && h.bc[b] == s->m->bc[b];
    if (!same) return fail(DVM_ERR_ARG, "the checkpoint was written for another mesh, velocity grid or precision");
    if (h.hybrid_fluid && !s->hybrid)
        return fail(DVM_ERR_ARG, "the checkpoint holds fluid cells: create the solver with params.hybrid = 1");
    if (net && !h.has_net) return fail(DVM_ERR_ARG, "the checkpoint holds no network");
    for (const Leaf &l : s->m->cells) {
        uint64_t key = 0;
        uint8_t level = 0;
        int32_t ijk[3];
        if (!f.read(&key, 8) || !f.read(&level, 1) || !f.read(ijk, 12))
            return fail(DVM_ERR_ARG, "checkpoint file is truncated");
        if (key != l.key || level != l.level || ijk[0] != l.i || ijk[1] != l.j || ijk[2] != l.k)
            return fail(DVM_ERR_ARG, "the checkpoint's leaf list differs from the solver's mesh");
    }
    // f in canonical order into the other state buffer, then into the current one
    void *stage = s->f[s->cur ^ 1];
    int rc = file_to_dev(f, stage, size_t(s->n) * size_t(s->nv) * (s->fp64 ? 8 : 4), st);
    if (rc) return rc;
    rc = dvm_f_from_canonical(s, stage, s->f[s->cur], stream);
    if (rc) return rc;
    rc = file_to_dev(f, s->mom, size_t(5) * size_t(s->n) * 8, st);
    if (!rc && h.hybrid) {
        if (s->hybrid) {
            rc = file_to_dev(f, solver_hybrid_prev(s), size_t(s->n), st);
        } else {
            std::vector<char> skip(size_t(s->n));
            if (!f.read(skip.data(), skip.size())) rc = fail(DVM_ERR_ARG, "checkpoint file is truncated");
        }
    }
    if (!rc && h.has_net) {
        if (net) {
            rc = file_to_dev(f, net->params, size_t(kMlpParams) * 4, st);
            if (!rc) rc = file_to_dev(f, net->m(), size_t(kMlpWeights) * 4, st);
            if (!rc) rc = file_to_dev(f, net->v(), size_t(kMlpWeights) * 4, st);
            if (!rc) net->t = h.net_t;
        } else {
            std::vector<char> skip(size_t(kMlpParams + 2 * kMlpWeights) * 4);
            if (!f.read(skip.data(), skip.size())) rc = fail(DVM_ERR_ARG, "checkpoint file is truncated");
        }
    }
    if (rc) return rc;
    const uint64_t want = f.sum.h;
    uint64_t got = 0;
    if (std::fread(&got, 1, 8, f.fp) != 8 || got != want)
        return fail(DVM_ERR_ARG, "checkpoint checksum mismatch: %s is damaged (the solver state is not valid)", path);
    s->steps = h.steps;
    s->hybrid_fluid = h.hybrid_fluid != 0;
    return DVM_OK;
}

}  // extern "C"
