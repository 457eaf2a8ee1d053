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
  * closed_half_flux() (the paper names the closed-form half-Maxwellian
    fluxes without printing them; pinned by quadrature of the defining
    integral and by the Euler flux identity):
    the half-range integral over xi_b > 0 or < 0 of xi_b (1, xi, |xi|^2/2)
    times the continuous Maxwellian of U; Hybrid(flux="closed") uses it on
    faces between two fluid cells in place of the discrete half-range sums
    (grid_half_flux()), faces next to a kinetic cell keep the sums.
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


def velocity_nodes(nv, vlo, vhi):
    """node velocities [3][N] in canonical order (x slowest) and the node volume"""
    d = [(vhi[a] - vlo[a]) / nv[a] for a in range(3)]
    axes = [vlo[a] + (np.arange(nv[a]) + 0.5) * d[a] for a in range(3)]
    X = np.meshgrid(*axes, indexing="ij")
    return np.stack([x.ravel() for x in X]), d[0] * d[1] * d[2]


def grid_half_flux(nv, vlo, vhi, U, b, positive):
    """node volume times the sum over the nodes with xi_b > 0 (positive) or
    xi_b < 0 of xi_b (1, xi, |xi|^2/2) Mt(U)"""
    m = maxwellian_of_moments(nv, vlo, vhi, U)
    xi, w = velocity_nodes(nv, vlo, vhi)
    sel = xi[b] > 0 if positive else xi[b] < 0
    x, mm = xi[:, sel], m[sel]
    psi = np.stack([np.ones(x.shape[1]), x[0], x[1], x[2], 0.5 * (x * x).sum(0)])
    return w * (psi * (x[b] * mm)).sum(1)


def closed_half_flux(U, b, positive):
    """integral over xi_b > 0 (positive) or xi_b < 0 of xi_b (1, xi,
    |xi|^2/2) M, M the Maxwellian of U = (rho, rho u, E).  Along b,
    xi_b = u_b + sqrt(T) t with t standard normal; the half-space is
    t > -s or t < -s (s = u_b / sqrt(T)) and its raw moments
    E[xi_b^k ; half] come from the truncated moments of t; the other two
    axes are full Gaussians (mean u_a, second moment u_a^2 + T)."""
    from scipy.special import erfc
    rho, u, T = primitive(np.asarray(U, np.float64)[:, None])
    rho, u, T = float(rho[0]), u[:, 0], float(T[0])
    sd = math.sqrt(T)
    s = u[b] / sd
    sgn = 1.0 if positive else -1.0
    q = 0.5 * erfc(-sgn * s / math.sqrt(2.0))              # P(half)
    phi = math.exp(-0.5 * s * s) / math.sqrt(2.0 * math.pi)
    t = [q, sgn * phi, q - sgn * s * phi, sgn * (s * s + 2.0) * phi]   # E[t^k ; half]
    m = [sum(math.comb(k, j) * u[b] ** (k - j) * sd ** j * t[j] for j in range(k + 1)) for k in range(4)]
    out = np.zeros(5)
    out[0] = rho * m[1]
    for a in range(3):
        out[1 + a] = rho * (m[2] if a == b else u[a] * m[1])
    trans = sum(u[a] * u[a] + T for a in range(3) if a != b)
    out[4] = 0.5 * rho * (m[3] + m[1] * trans)
    return out


class Hybrid:
    """Kinetic cells carry f, fluid cells carry U; the mask (1 = kinetic) is
    frozen for a step.  Switching: a cell that becomes kinetic starts from
    Mt(U); a cell that becomes fluid keeps the moments of its f."""

    def __init__(self, solver: O.Solver, params: O.OrParams, nv, vlo, vhi, flux="grid"):
        self.s = solver
        self.p = params
        self.nv, self.vlo, self.vhi = nv, vlo, vhi
        self.flux = flux
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
        U0 = self.U.copy()
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
        if self.flux == "closed":
            self._closed_faces(U0, dt)

    def _closed_faces(self, U0, dt):
        """On every face between two fluid cells replace the discrete
        half-range fluxes of the transport (U0: the states before the step)
        by the closed-form ones: U -= dt/h sum over such (sub)faces of
        sign * ((H_out - G_out) + (H_in - G_in)) / k, k the (sub)faces of the
        face, H closed form, G the grid sums, sign the outward normal."""
        t = self.s.mesh.tables()
        ty, nb, lev = t["type"], t["nbr"], t["level"]
        h0 = self.s.mesh.forest.h0
        args = (self.nv, self.vlo, self.vhi)
        for c in np.nonzero(~self.kinetic)[0]:
            acc = np.zeros(5)
            for f in range(6):
                b, side = f // 2, f % 2
                k = 4 if ty[c, f] == O.FACE_FINER else 1 if ty[c, f] in (O.FACE_SAME, O.FACE_COARSER) else 0
                for q in range(k):
                    e = nb[c, f, q]
                    if self.kinetic[e]:
                        continue
                    d_out = closed_half_flux(U0[:, c], b, side == 1) - grid_half_flux(*args, U0[:, c], b, side == 1)
                    d_in = closed_half_flux(U0[:, e], b, side == 0) - grid_half_flux(*args, U0[:, e], b, side == 0)
                    acc += (1.0 if side else -1.0) * (d_out + d_in) / k
            self.U[:, c] -= dt / (h0 / 2.0 ** int(lev[c])) * acc
