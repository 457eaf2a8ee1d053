"""CPU pins of the oracle's closed-form half-range Maxwellian fluxes
(oracle.sensor.closed_half_flux) and of the hybrid step that uses them on
faces between two fluid cells (Hybrid(flux="closed")).  The paper names
closed-form half-Maxwellian fluxes for the continuum cells without printing
them; the pins below are the defining integral (by quadrature), the Euler
flux identity, the u = 0 special case, the discrete sums' convergence, and
direct brute force of the fluid update on a tiny uniform mesh."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O
from oracle import sensor as S
from paper_1503_00707_amd import inputs as I

CASES = [(1.1, (0.4, -0.3, 0.2), 0.9), (0.7, (-1.3, 0.5, 0.0), 1.6), (2.0, (0.0, 0.0, 2.5), 0.4),
         (1.0, (3.0, -0.1, 0.7), 1.0)]


def _U(rho, u, T):
    u = np.asarray(u, float)
    return np.array([rho, rho * u[0], rho * u[1], rho * u[2], 0.5 * rho * (u @ u) + 1.5 * rho * T])


def _quadrature(rho, u, T, b, positive):
    """the defining integral: adaptive quadrature along xi_b over the half
    line, Gauss-Hermite (exact for these polynomial degrees) across"""
    gx, gw = np.polynomial.hermite_e.hermegauss(12)
    gw = gw / math.sqrt(2 * math.pi)
    a1, a2 = [a for a in range(3) if a != b]
    X1 = u[a1] + math.sqrt(T) * gx[:, None]
    X2 = u[a2] + math.sqrt(T) * gx[None, :]
    W = gw[:, None] * gw[None, :]

    def integrand(xb, comp):
        g = rho * math.exp(-(xb - u[b]) ** 2 / (2 * T)) / math.sqrt(2 * math.pi * T)
        xi = [None] * 3
        xi[b], xi[a1], xi[a2] = xb, X1, X2
        if comp == 0:
            psi = 1.0 + 0 * X1 * X2
        elif comp < 4:
            psi = xi[comp - 1] + 0 * X1 * X2
        else:
            psi = 0.5 * (xb * xb + X1 * X1 + X2 * X2)
        return xb * g * float((W * psi).sum())

    lo, hi = (0.0, np.inf) if positive else (-np.inf, 0.0)
    return np.array([integrate.quad(integrand, lo, hi, args=(k,), epsabs=1e-14, epsrel=1e-13, limit=200)[0]
                     for k in range(5)])


@pytest.mark.parametrize("case", CASES)
def test_closed_flux_is_the_half_range_integral(case):
    rho, u, T = case
    for b in range(3):
        for pos in (True, False):
            got = S.closed_half_flux(_U(rho, u, T), b, pos)
            want = _quadrature(rho, u, T, b, pos)
            scale = rho * (1 + abs(u[b]) + math.sqrt(T)) ** 3
            assert np.abs(got - want).max() <= 1e-11 * scale, (b, pos, got, want)


@pytest.mark.parametrize("case", CASES)
def test_both_halves_give_the_euler_flux(case):
    rho, u, T = case
    U = _U(rho, u, T)
    p, E = rho * T, U[4]
    for b in range(3):
        tot = S.closed_half_flux(U, b, True) + S.closed_half_flux(U, b, False)
        want = np.array([rho * u[b], *(rho * u[b] * np.asarray(u) + p * np.eye(3)[b]), u[b] * (E + p)])
        assert np.abs(tot - want).max() <= 1e-13 * max(1.0, np.abs(want).max())


def test_gas_at_rest_mass_flux_and_pressure():
    rho, T = 1.3, 0.8
    U = _U(rho, (0.0, 0.0, 0.0), T)
    for b in range(3):
        fp, fm = S.closed_half_flux(U, b, True), S.closed_half_flux(U, b, False)
        assert abs(fp[0] - rho * math.sqrt(T / (2 * math.pi))) <= 1e-15
        assert abs(fm[0] + fp[0]) <= 1e-15
        assert abs(fp[1 + b] - 0.5 * rho * T) <= 1e-15          # half the pressure each way
        assert abs(fp[4] - rho * T * math.sqrt(2 * T / math.pi)) <= 1e-14


def test_grid_sums_converge_to_the_closed_form():
    U = _U(1.1, (0.4, -0.3, 0.2), 0.9)
    errs = []
    for n in (16, 32):
        g = S.grid_half_flux((n, n, n), (-7.0,) * 3, (7.0,) * 3, U, 0, True)
        errs.append(np.abs(g - S.closed_half_flux(U, 0, True)).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] < 5e-3


def test_grid_half_flux_node_order_matches_the_moments():
    """the two halves of the grid sums add up to the full discrete flux
    w sum xi_b psi Mt, whose mass entry is the discrete momentum moment"""
    nv, lo, hi = (8, 8, 8), (-4.5,) * 3, (4.5,) * 3
    U = _U(1.1, (0.4, -0.3, 0.2), 0.9)
    mom = O.cell_moments(nv, lo, hi, S.maxwellian_of_moments(nv, lo, hi, U))
    for b in range(3):
        tot = S.grid_half_flux(nv, lo, hi, U, b, True) + S.grid_half_flux(nv, lo, hi, U, b, False)
        assert abs(tot[0] - mom[1 + b]) <= 1e-13


def _uniform_fluid(seed):
    f = I.uniform_forest((2, 2, 2), 0)
    m = O.Mesh(f)
    nv, lo, hi = (8, 8, 8), (-4.5,) * 3, (4.5,) * 3
    p = O.make_params(nv, lo, hi, tau_or_kn=0.1)
    s = O.Solver(m, p)
    rng = np.random.default_rng(seed)
    prim = np.stack([1 + 0.2 * rng.random(8), 0.3 * rng.standard_normal(8), 0.3 * rng.standard_normal(8),
                     0.3 * rng.standard_normal(8), 1 + 0.2 * rng.random(8)])
    s.init_maxwellian(prim)
    return f, m, p, s, nv, lo, hi


@pytest.mark.parametrize("seed", [0, 1])
def test_all_fluid_closed_step_is_the_direct_flux_sum(seed):
    """2^3 periodic cells (each face's neighbour across): the closed-form
    hybrid step of an all-fluid mask is U - dt/h sum over the 6 faces of
    sign * (H_out(U_c) + H_in(U_nb)), written out here cell by cell"""
    f, m, p, s, nv, lo, hi = _uniform_fluid(seed)
    t = m.tables()
    h = S.Hybrid(s, p, nv, lo, hi, flux="closed")
    h.set_mask(np.zeros(m.n_cells, bool))
    U0 = h.U.copy()
    dt = s.dt_cfl(0.5)
    h.step(dt)
    hc = f.h0
    for c in range(m.n_cells):
        acc = np.zeros(5)
        for face in range(6):
            b, side = face // 2, face % 2
            e = t["nbr"][c, face, 0]
            assert t["type"][c, face] == O.FACE_SAME
            acc += (1 if side else -1) * (S.closed_half_flux(U0[:, c], b, side == 1)
                                          + S.closed_half_flux(U0[:, e], b, side == 0))
        want = U0[:, c] - dt / hc * acc
        assert np.abs(h.U[:, c] - want).max() <= 1e-14 * np.abs(U0).max()


def test_closed_mixed_mask_conserves_globally_and_differs_from_grid():
    f = I.random_forest(4, (2, 2, 2), 2, 0.3)
    f = __import__("dataclasses").replace(f, level=O.balance(f)[0], ijk=O.balance(f)[1])
    m = O.Mesh(f)
    t = m.tables()
    nv, lo, hi = (8, 8, 8), (-4.5,) * 3, (4.5,) * 3
    p = O.make_params(nv, lo, hi, tau_mode=0, tau_or_kn=0.05)
    out = {}
    for flux in ("grid", "closed"):
        s = O.Solver(m, p)
        s.init_maxwellian(I.fields("sines", I.leaf_centres(f)[t["input"]], seed=31))
        dt = s.dt_cfl(0.5)
        h = S.Hybrid(s, p, nv, lo, hi, flux=flux)
        rng = np.random.default_rng(9)
        vol = (f.h0 / 2.0 ** t["level"].astype(float)) ** 3
        tot0 = (h.U * vol).sum(1)
        for _ in range(3):
            h.set_mask(rng.random(m.n_cells) < 0.4)
            h.step(dt)
        tot = (h.U * vol).sum(1)
        scale = np.array([tot0[0], tot0[0], tot0[0], tot0[0], tot0[4]])
        assert np.all(np.abs(tot - tot0) <= 1e-13 * scale), flux
        out[flux] = h.U
    d = np.abs(out["closed"] - out["grid"]).max()
    assert 1e-6 < d < 5e-2
