"""Pins of the sensor / training / hybrid oracle (oracle/sensor.py) against
closed forms, identities and finite differences (CPU only)."""
import dataclasses
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import oracle as O
from oracle import sensor as S
from paper_1503_00707_amd import inputs as I


def _balanced(forest):
    lev, ijk = O.balance(forest)
    return dataclasses.replace(forest, level=lev, ijk=ijk)


# --- network pieces ----------------------------------------------------------

def test_gelu_identities():
    x = np.linspace(-6, 6, 241)
    g = S.gelu(x)
    assert S.gelu(np.array([0.0]))[0] == 0.0
    # x Phi(x) - (-x) Phi(-x) = x (Phi(x) + Phi(-x)) = x
    assert np.abs((g - S.gelu(-x)) - x).max() <= 1e-14
    assert np.abs(S.gelu(np.array([40.0]))[0] - 40.0) <= 1e-12 and abs(S.gelu(np.array([-40.0]))[0]) <= 1e-300
    h = 1e-6
    fd = (S.gelu(x + h) - S.gelu(x - h)) / (2 * h)
    assert np.abs(fd - S.gelu_prime(x)).max() <= 1e-8


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    p = I.mlp_init(5).astype(np.float64)
    p[I.MLP_WEIGHTS:I.MLP_WEIGHTS + 10] = rng.normal(0, 0.3, 10)       # mean
    p[I.MLP_WEIGHTS + 10:] = rng.uniform(0.5, 2.0, 10)                  # std
    nb = I.MLP_WEIGHTS
    p[:nb] += rng.normal(0, 0.05, nb)  # non-zero biases too
    x = rng.normal(0, 1.0, (7, 10))
    y = (rng.random(7) < 0.4).astype(float)
    loss, g = S.loss_and_grad(p, x, y, pos_weight=3.0)
    h = 1e-6
    fd = np.zeros(nb)
    for k in range(nb):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd[k] = (S.loss_and_grad(pp, x, y, 3.0)[0] - S.loss_and_grad(pm, x, y, 3.0)[0]) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * max(np.abs(g).max(), 1e-3)


def test_bce_closed_forms_and_extremes():
    z = np.zeros(4)
    y = np.array([0.0, 1.0, 1.0, 0.0])
    loss, dz = S.bce_with_logits(z, y, pos_weight=2.5)
    assert loss == pytest.approx(math.log(2.0) * (1 + 2.5 + 2.5 + 1) / 4, rel=1e-15)
    assert np.allclose(dz, np.array([0.5, -2.5 * 0.5, -2.5 * 0.5, 0.5]) / 4, rtol=0, atol=1e-17)
    loss, dz = S.bce_with_logits(np.array([800.0, -800.0]), np.array([1.0, 0.0]))
    assert loss == 0.0 and np.all(np.isfinite(dz))
    loss, _ = S.bce_with_logits(np.array([800.0]), np.array([0.0]))
    assert loss == pytest.approx(800.0, rel=1e-15)


def test_adam_first_steps_closed_form():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = v = np.zeros(3)
    lr = 1e-2
    w1, m, v = S.adam_step(w, g, m, v, 1, lr)
    assert np.allclose(w1, w - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-16)
    # a constant gradient keeps the bias-corrected step at lr g / (|g| + eps)
    w2, m, v = S.adam_step(w1, g, m, v, 2, lr)
    assert np.allclose(w2 - w1, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


# --- features ----------------------------------------------------------------

def test_features_uniform_state_closed_form():
    f = I.uniform_forest((1, 1, 1), 2)
    m = O.Mesh(f)
    t = m.tables()
    n = m.n_cells
    rho, u, T = 1.3, np.array([0.2, -0.1, 0.4]), 0.8
    mom = np.zeros((5, n))
    mom[0] = rho
    mom[1:4] = (rho * u)[:, None]
    mom[4] = 0.5 * rho * (u * u).sum() + 1.5 * rho * T
    x = S.features(mom, t, f.h0, 1, 0.05)
    want = np.array([math.log(rho), *(u / math.sqrt(T)), math.log(T), 0, 0, 0, 0, 0])
    assert np.abs(x - want[None, :]).max() <= 1e-14


@pytest.mark.parametrize("seed", [0, 1])
def test_features_linear_density_exact_across_level_jumps(seed):
    """rho = a + b x: central differences over face-neighbour values with
    distances h, 3h/4 (FINER) and 3h/2 (COARSER) are exact in the interior"""
    bc = (I.OUTFLOW,) * 6
    f = _balanced(I.random_forest(seed, (2, 2, 2), 3, 0.3, bc))
    m = O.Mesh(f)
    t = m.tables()
    xc = I.leaf_centres(f)[t["input"]]
    a, b, T = 2.0, 0.7, 1.1
    rho = a + b * xc[:, 0]
    mom = np.zeros((5, m.n_cells))
    mom[0] = rho
    mom[4] = 1.5 * rho * T
    x = S.features(mom, t, f.h0, 0, 0.2)
    lam = 0.2 * math.sqrt(T)
    # both x faces inside the domain (any level jump); the y and z sides at the
    # cell's own x (SAME neighbours or domain faces), so the transverse
    # differences of a field that varies along x vanish
    ty = t["type"]
    interior = np.all(ty[:, 0:2] <= 2, axis=1) & np.all((ty[:, 2:6] == 0) | (ty[:, 2:6] >= 3), axis=1)
    jumps = interior & np.any((ty[:, 0:2] == 1) | (ty[:, 0:2] == 2), axis=1)
    assert interior.sum() > 10 and jumps.sum() > 2
    assert np.abs(x[interior, 5] - lam * b / rho[interior]).max() <= 1e-13
    assert np.abs(x[:, 6:10]).max() <= 1e-14  # u = 0, T uniform


# --- labels --------------------------------------------------------------------

def test_labels_zero_for_maxwellian_and_exact_for_moment_free_perturbation():
    nv, lo, hi = (8, 8, 8), (-4.5,) * 3, (4.5,) * 3
    mt = O.cell_maxwellian(nv, lo, hi, [1.2, 0.0, 0.0, 0.0, 0.9])
    g = np.stack(np.meshgrid(*[np.linspace(-4.5 + 0.5625, 4.5 - 0.5625, 8)] * 3, indexing="ij"), -1).reshape(-1, 3)
    delta = mt * (g[:, 0] ** 2 - g[:, 1] ** 2)  # zero mass, momentum and energy by symmetry
    eps = 1e-3
    f = np.stack([mt, 2.0 * mt, mt + eps * delta])
    r = S.labels(f, nv, lo, hi)
    assert r[0] <= 1e-13 and r[1] <= 1e-13  # the re-solved Mt agrees to rounding
    assert r[2] == pytest.approx(eps * np.linalg.norm(delta) / np.linalg.norm(mt), rel=1e-10)


# --- half-range fluxes and the hybrid step ------------------------------------

def test_half_range_mass_flux_converges_to_closed_form():
    """the discrete half-range flux w sum_{xi_x > 0} xi_x Mt tends to the
    continuum rho (sqrt(T / 2 pi) e^{-u^2 / 2T} + u/2 (1 + erf(u / sqrt(2T))))"""
    rho, ux, T = 1.1, 0.4, 0.9
    exact = rho * (math.sqrt(T / (2 * math.pi)) * math.exp(-ux * ux / (2 * T))
                   + 0.5 * ux * (1 + erf(ux / math.sqrt(2 * T))))
    errs = []
    for n in (16, 32):
        vmax = 7.0
        mt = O.cell_maxwellian((n, n, n), (-vmax,) * 3, (vmax,) * 3, [rho, ux, 0.0, 0.0, T])
        dv = 2 * vmax / n
        xi = -vmax + (np.arange(n) + 0.5) * dv
        m3 = mt.reshape(n, n, n)
        pos = xi > 0
        flux = dv ** 3 * (xi[pos, None, None] * m3[pos]).sum()
        errs.append(abs(flux - exact) / exact)
    # second order in dv (the integrand has a kink at xi_x = 0)
    assert errs[0] / errs[1] > 3.5 and errs[1] < 6e-3


def _hybrid_case(seed=2, tau=0.05):
    f = _balanced(I.random_forest(seed, (2, 2, 2), 2, 0.3))
    m = O.Mesh(f)
    t = m.tables()
    nv, lo, hi = (8, 8, 8), (-4.5,) * 3, (4.5,) * 3
    p = O.make_params(nv, lo, hi, tau_mode=0, tau_or_kn=tau)
    s = O.Solver(m, p)
    prim = I.fields("sines", I.leaf_centres(f)[t["input"]], seed=31)
    s.init_maxwellian(prim)
    return f, m, t, p, s, nv, lo, hi


def test_hybrid_all_kinetic_equals_plain_step_bitwise():
    f, m, t, p, s, nv, lo, hi = _hybrid_case()
    dt = s.dt_cfl(0.5)
    h = S.Hybrid(s, p, nv, lo, hi)
    f0 = s.get_f()
    for _ in range(3):
        h.step(dt)
    s2 = O.Solver(m, p)
    s2.set_f(f0)
    s2.step(dt, 3)
    assert np.array_equal(h.f, s2.get_f())


def test_hybrid_all_fluid_uniform_state_is_stationary():
    f = I.uniform_forest((2, 2, 2), 1)
    m = O.Mesh(f)
    nv, lo, hi = (8, 8, 8), (-4.5,) * 3, (4.5,) * 3
    p = O.make_params(nv, lo, hi, tau_or_kn=0.1)
    s = O.Solver(m, p)
    s.init_maxwellian(np.tile(np.array([[1.1], [0.3], [-0.2], [0.1], [0.95]]), (1, m.n_cells)))
    h = S.Hybrid(s, p, nv, lo, hi)
    U0 = h.U.copy()
    h.set_mask(np.zeros(m.n_cells, bool))
    for _ in range(4):
        h.step(s.dt_cfl(0.5))
    assert np.abs(h.U - U0).max() <= 1e-14 * np.abs(U0).max()


def test_hybrid_mixed_mask_conserves_globally():
    f, m, t, p, s, nv, lo, hi = _hybrid_case(seed=4)
    dt = s.dt_cfl(0.5)
    h = S.Hybrid(s, p, nv, lo, hi)
    rng = np.random.default_rng(9)
    vol = (f.h0 / 2.0 ** t["level"].astype(float)) ** 3
    tot0 = (h.U * vol).sum(1)
    for _ in range(3):
        h.set_mask(rng.random(m.n_cells) < 0.5)
        h.step(dt)
    tot = (h.U * vol).sum(1)
    scale = np.array([tot0[0], tot0[0], tot0[0], tot0[0], tot0[4]])
    assert np.all(np.abs(tot - tot0) <= 1e-13 * scale)
