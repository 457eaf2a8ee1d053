"""Training and evaluation of the continuum-breakdown sensor on the GPU.

Data: seeded runs of the DVM step on the 16^3 periodic mesh with 8^3
velocities on [-4.5, 4.5]^3, each run's rho, u, T perturbed by random
sinusoids (inputs.fields("sensor_runs")) and its relaxation time drawn
log-uniform in [TAU_LO, 1] (near-continuum to rarefied); at every step the
features of the moments (dvm_features) and the non-equilibrium measure r = |f - Mt| / |Mt|
(dvm_labels) of a seeded subset of cells are kept, the features before a
step and r after it; a cell is "kinetic" when r > theta, theta calibrated
against the hybrid's error bar.  Training: dvm_mlp_train_step (class-weighted BCE, Adam)
over shuffled mini-batches.  Evaluation: the hybrid step driven by the
sensor against full DVM on the same flow (moment error in the norm of
max rho, max rho sqrt(max T), max E) and its time.

Everything that computes runs in the HIP library; this module only
selects, batches and times.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import dvm as D
from . import inputs as I

LABEL_THRESHOLD = 0.05   # default; train(threshold=...) takes the calibrated one
ERROR_BAR = 1e-3         # moment error of the hybrid against full DVM (max over the run's end state)
NV, VMAX = 8, 4.5
TAU_LO = 0.001           # smallest relaxation time of the training and calibration runs
TRAINED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sensor_net.json")


def c1_mesh(level=4):
    return I.uniform_forest((1, 1, 1), level, 1.0)


def generate(runs, seed0=0, steps=20, keep=256, precision=D.PREC_FP32, log=None):
    """features [N, 10] and labels r [N] (torch, on the GPU) of `runs` seeded runs"""
    import torch
    forest = c1_mesh()
    mesh = D.Mesh(forest)
    t = mesh.tables()
    xc = I.leaf_centres(forest)[t["input"]]
    xs, rs = [], []
    for k in range(runs):
        seed = seed0 + k
        tau = I.sensor_run_tau(seed, lo=TAU_LO)
        p = D.make_params(NV, VMAX, precision=precision, tau_or_kn=tau)
        s = D.Solver(mesh, p)
        s.init_maxwellian(I.fields("sensor_runs", xc, seed=seed))
        dt = s.dt(0.5)
        rng = np.random.default_rng([seed, 11])
        for _ in range(steps):
            # features of the state before the step, the label of the state after it:
            # a cell can be fluid for this step if the kinetic run's next state is
            # near its Maxwellian (otherwise turning it kinetic again loses that part)
            idx = torch.as_tensor(rng.choice(s.n, size=min(keep, s.n), replace=False), device="cuda")
            xs.append(s.features()[idx])
            s.step(1, dt=dt)
            rs.append(s.labels()[idx])
        if log and (k + 1) % max(1, runs // 10) == 0:
            log(f"[sensor] generated {k + 1}/{runs} runs")
    return torch.cat(xs), torch.cat(rs)


def train(x, r, epochs=10, batch=4096, lr=3e-3, seed=0, log=None, threshold=LABEL_THRESHOLD):
    """a network trained on (x, r > threshold); returns (net, per-epoch mean loss, pos_weight)"""
    import torch
    y = (r > threshold).float()
    n_pos = float(y.sum().item())
    n = x.shape[0]
    pos_weight = max(1.0, (n - n_pos) / max(n_pos, 1.0))
    net = D.MLP(I.mlp_init(seed), max_batch=batch)
    net.set_normalization(x)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device="cuda")
        losses = []
        lr_ep = lr * 0.5 * (1.0 + math.cos(math.pi * ep / epochs))  # cosine decay per epoch
        for b0 in range(0, n - batch + 1, batch):
            sel = perm[b0:b0 + batch]
            net.train_step(x[sel], y[sel], lr=lr_ep, pos_weight=pos_weight)
            if (b0 // batch) % 64 == 0:
                losses.append(net.grads_and_loss()[1])
        hist.append(float(np.mean(losses)))
        if log:
            log(f"[sensor] epoch {ep + 1}/{epochs}: loss {hist[-1]:.4f}")
    return net, hist, pos_weight


def accuracy(net, x, r, threshold=LABEL_THRESHOLD):
    """(accuracy, recall of kinetic cells, false-kinetic rate) of the matrix-core forward"""
    y = (r > threshold).cpu().numpy()
    z = net.forward(x, mode=1).cpu().numpy()
    pred = z > 0
    acc = float((pred == y).mean())
    recall = float(pred[y].mean()) if y.any() else float("nan")
    false_kin = float(pred[~y].mean()) if (~y).any() else float("nan")
    return acc, recall, false_kin


def _moment_error(m, ref):
    rho = ref[0]
    u = ref[1:4] / rho
    T = (2 * ref[4] / rho - (u * u).sum(0)) / 3
    su = rho.max() * math.sqrt(T.max())
    scale = np.array([rho.max(), su, su, su, ref[4].max()])
    return float((np.abs(m - ref).max(axis=1) / scale).max())


class HybridGraph:
    """Two steps of "sensor on the current moments, then one hybrid step under
    that mask" recorded once into a HIP graph (through torch's graph capture
    of the library's launches on the current stream) and replayed: the
    buffer parity returns to where it started after two steps, so one
    recording serves every replay.  net None: Kn_GLL > kappa."""

    def __init__(self, solver, net, kappa, dt):
        import torch
        self.torch = torch
        self.g = torch.cuda.CUDAGraph()
        self.masks = []
        torch.cuda.synchronize()
        with torch.cuda.graph(self.g):
            for _ in range(2):
                mask, _ = solver.sensor(net, kappa) if net is not None else solver.sensor(None, kappa)
                solver.hybrid_step(mask, n=1, dt=dt)
                self.masks.append(mask)

    def replay(self):
        self.g.replay()


class PlainGraph:
    """Two plain DVM steps recorded into a HIP graph (the plain side of a timing comparison)."""

    def __init__(self, solver, dt):
        import torch
        self.g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(self.g):
            solver.step(2, dt=dt)

    def replay(self):
        self.g.replay()


def evaluate(net, kappa=None, fields="sine_rho", field_args=None, tau=0.1, steps=20, precision=D.PREC_FP32,
             level=4, nv=NV, vmax=VMAX, graph=False, fluid_flux=D.FLUX_GRID):
    """hybrid (sensor every step) vs full DVM on one flow of the periodic
    unit cube at 2^level cells per side (4: the C1 mesh): dict with the moment
    error, mean kinetic fraction, and both step times.  graph: both sides
    replay two-step HIP graphs (steps must be even).  fluid_flux: the
    hybrid's fluxes between fluid cells (discrete sums or closed form)."""
    import torch
    field_args = {"a": 0.1} if field_args is None else field_args
    forest = c1_mesh(level)
    mesh = D.Mesh(forest)
    t = mesh.tables()
    prim = I.fields(fields, I.leaf_centres(forest)[t["input"]], **field_args)
    p = D.make_params(nv, vmax, precision=precision, tau_or_kn=tau, hybrid=True, fluid_flux=fluid_flux)
    full = D.Solver(mesh, p)
    full.init_maxwellian(prim)
    hyb = D.Solver(mesh, p)
    hyb.init_maxwellian(prim)
    dt = full.dt(0.5)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if graph:
        assert steps % 2 == 0
        pg = PlainGraph(full, dt)
        hg = HybridGraph(hyb, net, 0.0 if kappa is None else kappa, dt)
    e0.record()
    if graph:
        for _ in range(steps // 2):
            pg.replay()
    else:
        full.step(steps, dt=dt)
    e1.record()
    torch.cuda.synchronize()
    t_full = e0.elapsed_time(e1)
    e0.record()
    if graph:
        for _ in range(steps // 2):
            hg.replay()
    else:
        for _ in range(steps):
            mask, _ = hyb.sensor(net) if kappa is None else hyb.sensor(None, kappa)
            hyb.hybrid_step(mask, n=1, dt=dt)
    e1.record()
    torch.cuda.synchronize()
    t_hyb = e0.elapsed_time(e1)
    # the kinetic fraction from an eager replica, outside the timed region; with
    # graphs the replica must also end in the graph-replayed state, bitwise
    rep = D.Solver(mesh, p)
    rep.init_maxwellian(prim)
    fracs = []
    for _ in range(steps):
        mask, _ = rep.sensor(net) if kappa is None else rep.sensor(None, kappa)
        rep.hybrid_step(mask, n=1, dt=dt)
        fracs.append(mask.float().mean())
    frac = float(torch.stack(fracs).mean().item())
    mh = hyb.moments().cpu().numpy()
    same = bool(np.array_equal(mh, rep.moments().cpu().numpy()))
    if not same:
        raise RuntimeError("graph replay of the hybrid step differs from the eager steps")
    err = _moment_error(mh, full.moments().cpu().numpy())
    return dict(error=err, kinetic_fraction=frac, ms_full=t_full / steps, ms_hybrid=t_hyb / steps,
                speedup=t_full / t_hyb, graph=bool(graph))


# ---------------------------------------------------------------------------
# calibration against the error bar: full DVM is the reference
# ---------------------------------------------------------------------------

def flow(seed, tau=None):
    """(recipe, field arguments, tau) of a sensor run; seed None: the C1 flow
    (rho = 1 + 0.1 sin 2 pi x, tau = 0.1, or the given tau)"""
    if seed is None:
        return "sine_rho", {"a": 0.1}, 0.1 if tau is None else float(tau)
    return "sensor_runs", {"seed": int(seed)}, I.sensor_run_tau(int(seed), lo=TAU_LO) if tau is None else float(tau)


def lockstep(seed, policies, steps=20, level=4, nv=NV, vmax=VMAX, precision=D.PREC_FP32, tau=None):
    """Full DVM and one hybrid solver per policy, advanced together on one
    flow; each step a policy gives the frozen mask of its hybrid from the
    states before the step.  Policies: ("labels", theta): r > theta of the
    full-DVM state (the mask a perfect sensor of that label would give);
    ("kn", kappa): Kn_GLL > kappa of the hybrid's own moments; ("net", net):
    the network on the hybrid's own moments; ("fluid",), ("kinetic",).
    Returns per policy (moment error after `steps`, mean kinetic fraction)."""
    import torch
    recipe, args, tau = flow(seed, tau)
    forest = c1_mesh(level)
    mesh = D.Mesh(forest)
    t = mesh.tables()
    prim = I.fields(recipe, I.leaf_centres(forest)[t["input"]], **args)
    p = D.make_params(nv, vmax, precision=precision, tau_or_kn=tau, hybrid=True)
    full = D.Solver(mesh, p)
    full.init_maxwellian(prim)
    hyb = []
    for _ in policies:
        h = D.Solver(mesh, p)
        h.init_maxwellian(prim)
        hyb.append(h)
    dt = full.dt(0.5)
    kin = [0.0] * len(policies)
    ones = torch.ones(full.n, dtype=torch.uint8, device="cuda")
    for _ in range(steps):
        full.step(1, dt=dt)
        r = None
        for k, (pol, h) in enumerate(zip(policies, hyb)):
            if pol[0] == "labels":
                # the label the sensor is trained on: the kinetic run's state after this step
                r = full.labels() if r is None else r
                mask = (r > pol[1]).to(torch.uint8)
            elif pol[0] == "kn":
                mask, _ = h.sensor(None, pol[1])
            elif pol[0] == "net":
                mask, _ = h.sensor(pol[1])
            elif pol[0] == "fluid":
                mask = 0 * ones
            else:
                mask = ones
            kin[k] += float(mask.float().mean().item()) / steps
            h.hybrid_step(mask, n=1, dt=dt)
    ref = full.moments().cpu().numpy()
    return [(_moment_error(h.moments().cpu().numpy(), ref), kin[k]) for k, h in enumerate(hyb)]


def calibrate(make_policy, values, seeds, margin=0.75, log=None, name="value"):
    """the value (ordered from most to fewest kinetic cells) with the fewest
    kinetic cells whose hybrid stays within margin * ERROR_BAR on every seed;
    returns (value, table of (value, max error, mean kinetic fraction))"""
    table = []
    policies = [make_policy(v) for v in values]
    res = [lockstep(sd, policies) for sd in seeds]
    best = values[0]
    for k, v in enumerate(values):
        err = max(r[k][0] for r in res)
        frac = float(np.mean([r[k][1] for r in res]))
        table.append((v, err, frac))
        if log:
            log(f"[sensor] {name} {v:.4g}: max error {err:.3e}, kinetic fraction {frac:.3f}")
        if err <= margin * ERROR_BAR:
            best = v
    return best, table


def net_with_logit_shift(net, shift):
    """the same network deciding "kinetic" at logit > shift (b3 lowered by shift)"""
    p = net.params.detach().cpu().numpy().copy()
    p[I.MLP_WEIGHTS - 1] -= shift
    return D.MLP(p, max_batch=16)


def save_trained(path, net, meta):
    meta = dict(meta)
    meta["params"] = [float(v) for v in net.params.detach().cpu().numpy()]
    with open(path, "w") as fh:
        json.dump(meta, fh)


def load_trained(path=TRAINED):
    """(network, metadata) of the committed trained sensor"""
    with open(path) as fh:
        meta = json.load(fh)
    p = np.asarray(meta.pop("params"), np.float32)
    return D.MLP(p, max_batch=16), meta


def build_trained(runs=2000, epochs=10, calib_seeds=range(0, 160), eval_seeds=range(10000, 10064), log=None,
                  path=TRAINED):
    """The committed sensor: calibrate the label threshold against the error
    bar (exact labels as masks), generate the training data, train, calibrate
    the decision threshold of the network and the Kn_GLL baseline's kappa on
    the same calibration runs, evaluate on held-out flows; write `path`."""
    t0 = time.time()
    thetas = [0.0005, 0.001, 0.00125, 0.0015, 0.00175, 0.002, 0.003]
    theta, th_table = calibrate(lambda v: ("labels", v), thetas, calib_seeds, log=log, name="label theta")
    x, r = generate(runs, seed0=0, log=log)
    if log:
        log(f"[sensor] {x.shape[0]} samples, kinetic at theta {theta}: {float((r > theta).float().mean()):.3f} "
            f"({time.time() - t0:.0f}s)")
    net, hist, pw = train(x, r, epochs=epochs, log=log, threshold=theta)
    shifts = [-2.0, -1.0, -0.5, 0.0, 0.5, 1.0, 1.5, 2.0, 3.0]
    shift, sh_table = calibrate(lambda v: ("net", net_with_logit_shift(net, v)), shifts, calib_seeds, log=log,
                                name="logit shift")
    tuned = net_with_logit_shift(net, shift)
    kappas = [0.001, 0.002, 0.004, 0.008, 0.016, 0.032, 0.064, 0.128, 0.256]
    kappa, kn_table = calibrate(lambda v: ("kn", v), kappas, calib_seeds, log=log, name="Kn_GLL kappa")
    xv, rv = generate(len(eval_seeds), seed0=eval_seeds[0])
    acc = accuracy(tuned, xv, rv, threshold=theta)
    meta = dict(label_threshold=theta, logit_shift=shift, kn_gll_kappa=kappa, error_bar=ERROR_BAR,
                tau_range=[TAU_LO, 1.0], runs=runs, epochs=epochs, samples=int(x.shape[0]), pos_weight=pw, loss=hist,
                calibration_seeds=[int(calib_seeds[0]), int(calib_seeds[-1])],
                label_threshold_table=th_table, logit_shift_table=sh_table, kappa_table=kn_table,
                heldout_accuracy=acc[0], heldout_recall=acc[1], heldout_false_kinetic=acc[2],
                build_seconds=time.time() - t0)
    save_trained(path, tuned, meta)
    return tuned, meta


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--runs", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--eval-runs", type=int, default=64)
    ap.add_argument("--build", action="store_true",
                    help="calibrate, train and write the committed sensor (sensor_net.json)")
    ap.add_argument("--out", default=TRAINED)
    ap.add_argument("--evaluate", action="store_true",
                    help="the committed sensor's hybrid against plain DVM on one flow (graphs on both sides)")
    ap.add_argument("--level", type=int, default=4, help="--evaluate: 2^level cells per side")
    ap.add_argument("--nv", type=int, default=NV, help="--evaluate: velocities per axis")
    ap.add_argument("--vmax", type=float, default=VMAX, help="--evaluate: velocity box half-width")
    ap.add_argument("--tau", type=float, default=0.1, help="--evaluate: relaxation time")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)
    if args.evaluate:
        net, _ = load_trained()
        r = evaluate(net, tau=args.tau, level=args.level, nv=args.nv, vmax=args.vmax, graph=True)
        print(json.dumps(r), flush=True)
        return r
    if args.build:
        _, meta = build_trained(runs=args.runs, epochs=args.epochs, log=log, path=args.out)
        print(json.dumps({k: v for k, v in meta.items() if not k.endswith("_table")}), flush=True)
        return meta
    t0 = time.time()
    x, r = generate(args.runs, seed0=0, log=log)
    log(f"[sensor] {x.shape[0]} samples, {float((r > LABEL_THRESHOLD).float().mean()):.3f} kinetic, "
        f"{time.time() - t0:.1f}s")
    net, hist, pw = train(x, r, epochs=args.epochs, log=log)
    xv, rv = generate(args.eval_runs, seed0=10000)
    acc = accuracy(net, xv, rv)
    out = dict(samples=int(x.shape[0]), pos_weight=pw, loss=hist, heldout_accuracy=acc[0], heldout_recall=acc[1],
               heldout_false_kinetic=acc[2], c1=evaluate(net))
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
