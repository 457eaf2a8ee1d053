"""Training and evaluation of the continuum-breakdown sensor on the GPU.

Data: seeded runs of the DVM step on the 16^3 periodic mesh with 8^3
velocities on [-4.5, 4.5]^3, each run's rho, u, T perturbed by random
sinusoids (inputs.fields("sensor_runs")) and its relaxation time drawn
log-uniform in [0.01, 1]; at every step the features of the moments
(dvm_features) and the non-equilibrium measure r = |f - Mt| / |Mt|
(dvm_labels) of a seeded subset of cells are kept; a cell is "kinetic"
when r > 0.05.  Training: dvm_mlp_train_step (class-weighted BCE, Adam)
over shuffled mini-batches.  Evaluation: the hybrid step driven by the
sensor against full DVM on the same flow (moment error in the norm of
max rho, max rho sqrt(max T), max E) and its time.

Everything that computes runs in the HIP library; this module only
selects, batches and times.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import dvm as D
from . import inputs as I

LABEL_THRESHOLD = 0.05
NV, VMAX = 8, 4.5


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
        tau = I.sensor_run_tau(seed)
        p = D.make_params(NV, VMAX, precision=precision, tau_or_kn=tau)
        s = D.Solver(mesh, p)
        s.init_maxwellian(I.fields("sensor_runs", xc, seed=seed))
        dt = s.dt(0.5)
        rng = np.random.default_rng([seed, 11])
        for _ in range(steps):
            s.step(1, dt=dt)
            idx = torch.as_tensor(rng.choice(s.n, size=min(keep, s.n), replace=False), device="cuda")
            xs.append(s.features()[idx])
            rs.append(s.labels()[idx])
        if log and (k + 1) % max(1, runs // 10) == 0:
            log(f"[sensor] generated {k + 1}/{runs} runs")
    return torch.cat(xs), torch.cat(rs)


def train(x, r, epochs=10, batch=4096, lr=3e-3, seed=0, log=None):
    """a network trained on (x, r > threshold); returns (net, per-epoch mean loss, pos_weight)"""
    import torch
    y = (r > LABEL_THRESHOLD).float()
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


def accuracy(net, x, r):
    """(accuracy, recall of kinetic cells, false-kinetic rate) of the matrix-core forward"""
    y = (r > LABEL_THRESHOLD).cpu().numpy()
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


def evaluate(net, kappa=None, fields="sine_rho", field_args=None, tau=0.1, steps=20, precision=D.PREC_FP32,
             level=4, nv=NV, vmax=VMAX):
    """hybrid (sensor every step) vs full DVM on one flow of the periodic
    unit cube at 2^level cells per side (4: the C1 mesh): dict with the moment
    error, mean kinetic fraction, and both step times"""
    import torch
    field_args = {"a": 0.1} if field_args is None else field_args
    forest = c1_mesh(level)
    mesh = D.Mesh(forest)
    t = mesh.tables()
    prim = I.fields(fields, I.leaf_centres(forest)[t["input"]], **field_args)
    p = D.make_params(nv, vmax, precision=precision, tau_or_kn=tau, hybrid=True)
    full = D.Solver(mesh, p)
    full.init_maxwellian(prim)
    hyb = D.Solver(mesh, p)
    hyb.init_maxwellian(prim)
    dt = full.dt(0.5)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    full.step(steps, dt=dt)
    e1.record()
    torch.cuda.synchronize()
    t_full = e0.elapsed_time(e1)
    fracs = []
    e0.record()
    for _ in range(steps):
        mask, _ = hyb.sensor(net) if kappa is None else hyb.sensor(None, kappa)
        hyb.hybrid_step(mask, n=1, dt=dt)
        fracs.append(mask)
    e1.record()
    torch.cuda.synchronize()
    t_hyb = e0.elapsed_time(e1)
    frac = float(torch.stack(fracs).float().mean().item())
    err = _moment_error(hyb.mom.cpu().numpy(), full.mom.cpu().numpy())
    return dict(error=err, kinetic_fraction=frac, ms_full=t_full / steps, ms_hybrid=t_hyb / steps,
                speedup=t_full / t_hyb)


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--runs", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--eval-runs", type=int, default=64)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)
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
