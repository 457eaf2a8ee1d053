"""FP64 oracle of the learned continuum-breakdown sensor, its training and the
kinetic/fluid hybrid step -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module.  Plain NumPy in float64 (the hybrid step drives the C oracle of
dvm_oracle.c for transport, Maxwellians and collisions); nothing here is
shared with the HIP library.

What it defines (the paper's hybrid solver couples kinetic and continuum
cells, sections 2-3; the sensor network, its features and its training are
the readings stated below):
  * features(): per cell, from the conserved moments and face-neighbour
    means, x = [ln rho, u/sqrt(T) (3), ln T, lambda |grad rho|/rho,
    lambda |grad u_b|/sqrt(T) (3), lambda |grad T|/T], lambda = tau sqrt(T);
    gradients by central differences over the face-neighbour values (the
    mean of the four leaves of a FINER face) with centre distances h (SAME
    and domain faces, where the cell's own value is used), 3h/4 (FINER) and
    3h/2 (COARSER).
  * mlp_forward()/mlp_backward(): 10-64-64-1, exact GELU (erf form), inputs
    standardised by a stored mean and standard deviation.
  * bce_with_logits(): class-weighted binary cross-entropy on the logit.
  * adam_step(): Adam with bias correction (beta = 0.9, 0.999, eps = 1e-8).
  * labels(): r = |f - Mt|_2 / |Mt|_2 over the velocity nodes, Mt the
    corrected Maxwellian (eq. 6) of the cell's own moments.
  * hybrid_step(): one step with a frozen mask.  Kinetic cells carry f,
    fluid cells carry U = (rho, rho u, E).  The state seen by the transport
    is g = f (kinetic) or Mt(U) (fluid); g is transported by eq. (2); a
    kinetic cell then relaxes (BGK to the eq. 6 Maxwellian), a fluid cell
    keeps only the moments of its transported g, which is the kinetic
    flux-vector-splitting update U - dt/V sum_faces A (H+(g_own) + H-(g_up))
    with the half-range fluxes of the discrete velocity set.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

FACE_SAME, FACE_COARSER, FACE_FINER = 0, 1, 2


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------

def primitive(mom):
    """(rho, u, T) from (rho, rho u, E); E = rho |u|^2 / 2 + 3 rho T / 2."""
    rho = mom[0]
    u = mom[1:4] / rho
    T = (2.0 * mom[4] / rho - (u * u).sum(0)) / 3.0
    return rho, u, T


def tau_of(rho, T, tau_mode, tau_or_kn):
    if tau_mode == 0:
        return np.full_like(rho, tau_or_kn)
    return tau_or_kn / (rho * np.sqrt(T))  # hard sphere


def _side_value(q, tables, h, c, f):
    """value and centre distance of the neighbour across face f of cell c"""
    ty = int(tables["type"][c, f])
    nb = tables["nbr"][c, f]
    if ty == FACE_SAME:
        return q[nb[0]], h
    if ty == FACE_COARSER:
        return q[nb[0]], 1.5 * h
    if ty == FACE_FINER:
        return 0.25 * (q[nb[0]] + q[nb[1]] + q[nb[2]] + q[nb[3]]), 0.75 * h
    return q[c], h  # domain face: the cell's own value


def gradient_norm(q, tables, h0):
    n = q.shape[0]
    out = np.zeros(n)
    for c in range(n):
        h = h0 / 2.0 ** int(tables["level"][c])
        s = 0.0
        for b in range(3):
            qm, dm = _side_value(q, tables, h, c, 2 * b)
            qp, dp = _side_value(q, tables, h, c, 2 * b + 1)
            d = (qp - qm) / (dm + dp)
            s += d * d
        out[c] = math.sqrt(s)
    return out


def features(mom, tables, h0, tau_mode, tau_or_kn):
    rho, u, T = primitive(mom)
    lam = tau_of(rho, T, tau_mode, tau_or_kn) * np.sqrt(T)
    sT = np.sqrt(T)
    x = np.zeros((rho.shape[0], 10))
    x[:, 0] = np.log(rho)
    x[:, 1:4] = (u / sT).T
    x[:, 4] = np.log(T)
    x[:, 5] = lam * gradient_norm(rho, tables, h0) / rho
    for b in range(3):
        x[:, 6 + b] = lam * gradient_norm(u[b], tables, h0) / sT
    x[:, 9] = lam * gradient_norm(T, tables, h0) / T
    return x


def kn_gll(x):
    """baseline sensor value: the largest gradient-length Knudsen number"""
    return x[:, 5:10].max(axis=1)


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------

IN, HID = 10, 64


def unpack(p):
    p = np.asarray(p, np.float64)
    o = 0

    def take(k, shape):
        nonlocal o
        a = p[o:o + k].reshape(shape)
        o += k
        return a
    w1 = take(HID * IN, (HID, IN))
    b1 = take(HID, (HID,))
    w2 = take(HID * HID, (HID, HID))
    b2 = take(HID, (HID,))
    w3 = take(HID, (HID,))
    b3 = take(1, (1,))
    mean = take(IN, (IN,))
    std = take(IN, (IN,))
    return dict(w1=w1, b1=b1, w2=w2, b2=b2, w3=w3, b3=b3, mean=mean, std=std)


def pack_grads(g):
    return np.concatenate([g["w1"].ravel(), g["b1"], g["w2"].ravel(), g["b2"], g["w3"], g["b3"]])


def gelu(z):
    from scipy.special import erf
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def mlp_forward(p, x):
    """logits z[n] and the intermediate values for the backward pass"""
    P = unpack(p)
    xs = (np.asarray(x, np.float64) - P["mean"]) / P["std"]
    z1 = xs @ P["w1"].T + P["b1"]
    h1 = gelu(z1)
    z2 = h1 @ P["w2"].T + P["b2"]
    h2 = gelu(z2)
    z = h2 @ P["w3"] + P["b3"][0]
    return z, dict(xs=xs, z1=z1, h1=h1, z2=z2, h2=h2)


def mlp_backward(p, cache, dz):
    """gradients of sum_i dz_i z_i with respect to the weights"""
    P = unpack(p)
    g = {}
    g["w3"] = dz @ cache["h2"]
    g["b3"] = np.array([dz.sum()])
    d2 = np.outer(dz, P["w3"]) * gelu_prime(cache["z2"])
    g["w2"] = d2.T @ cache["h1"]
    g["b2"] = d2.sum(0)
    d1 = (d2 @ P["w2"]) * gelu_prime(cache["z1"])
    g["w1"] = d1.T @ cache["xs"]
    g["b1"] = d1.sum(0)
    return g


def bce_with_logits(z, y, pos_weight=1.0):
    """mean class-weighted BCE and its derivative with respect to z"""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    w = np.where(y > 0.5, pos_weight, 1.0)
    loss = w * (np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z))))
    ez = np.exp(-np.abs(z))
    sig = np.where(z >= 0, 1.0 / (1.0 + ez), ez / (1.0 + ez))
    return loss.mean(), w * (sig - y) / z.shape[0]


def loss_and_grad(p, x, y, pos_weight=1.0):
    z, cache = mlp_forward(p, x)
    loss, dz = bce_with_logits(z, y, pos_weight)
    return loss, pack_grads(mlp_backward(p, cache, dz))


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """one Adam update of the weights w (t counts from 1); returns new (w, m, v)"""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# labels and the hybrid step
# ---------------------------------------------------------------------------

def labels(f, nv, vlo, vhi):
    """r = |f - Mt|_2 / |Mt|_2 per cell"""
    r = np.zeros(f.shape[0])
    for c in range(f.shape[0]):
        mom = O.cell_moments(nv, vlo, vhi, f[c])
        rho, u, T = primitive(mom[:, None])
        mt = O.cell_maxwellian(nv, vlo, vhi, [rho[0], u[0, 0], u[1, 0], u[2, 0], T[0]])
        r[c] = np.linalg.norm(f[c] - mt) / np.linalg.norm(mt)
    return r


def maxwellian_of_moments(nv, vlo, vhi, U):
    rho, u, T = primitive(np.asarray(U, np.float64)[:, None])
    return O.cell_maxwellian(nv, vlo, vhi, [rho[0], u[0, 0], u[1, 0], u[2, 0], T[0]])


class Hybrid:
    """Kinetic cells carry f, fluid cells carry U; the mask (1 = kinetic) is
    frozen for a step.  Switching: a cell that becomes kinetic starts from
    Mt(U); a cell that becomes fluid keeps the moments of its f."""

    def __init__(self, solver: O.Solver, params: O.OrParams, nv, vlo, vhi):
        self.s = solver
        self.p = params
        self.nv, self.vlo, self.vhi = nv, vlo, vhi
        self.f = solver.get_f()
        self.U = solver.moments()
        self.kinetic = np.ones(self.f.shape[0], bool)

    def set_mask(self, mask):
        mask = np.asarray(mask, bool)
        for c in np.nonzero(mask & ~self.kinetic)[0]:  # fluid -> kinetic
            self.f[c] = maxwellian_of_moments(self.nv, self.vlo, self.vhi, self.U[:, c])
        for c in np.nonzero(~mask & self.kinetic)[0]:  # kinetic -> fluid
            self.U[:, c] = O.cell_moments(self.nv, self.vlo, self.vhi, self.f[c])
        self.kinetic = mask.copy()

    def step(self, dt):
        g = self.f.copy()
        for c in np.nonzero(~self.kinetic)[0]:
            g[c] = maxwellian_of_moments(self.nv, self.vlo, self.vhi, self.U[:, c])
        self.s.set_f(g)
        self.s.transport(dt)
        fs = self.s.get_f()
        for c in range(fs.shape[0]):
            if self.kinetic[c]:
                rc, out = O.cell_collide(self.p, dt, fs[c])
                if rc:
                    raise RuntimeError(f"collision failed in cell {c}: {rc}")
                self.f[c] = out
                self.U[:, c] = O.cell_moments(self.nv, self.vlo, self.vhi, out)
            else:
                self.U[:, c] = O.cell_moments(self.nv, self.vlo, self.vhi, fs[c])
