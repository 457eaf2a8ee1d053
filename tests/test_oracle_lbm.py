"""Pins of the oracle's lattice Boltzmann subset (section 4: D3Q19 and D3Q27
as subsets of the DVM velocity grid, BGK collision toward the second-order
equilibrium) against what the lattice and the mathematics fix: the weights'
isotropy up to fourth order, the equilibrium's moments (mass, momentum and
the momentum flux rho cs^2 I + rho u u), conservation by the collision, the
homogeneous relaxation closed form, a uniform equilibrium at rest and in
motion stationary on an octree, global conservation on a periodic octree,
and the corner populations of D3Q19 staying empty."""
import dataclasses
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_00707_amd import inputs as I

C = np.array(list(itertools.product((-1.0, 0.0, 1.0), repeat=3)))  # canonical order of the 3^3 grid
CS2 = 1.0 / 3.0


def one_cell(q, tau=0.7, collision=4):
    m = O.Mesh(I.uniform_forest((1, 1, 1), 0))
    return m, O.Solver(m, O.lbm_params(q, tau, collision=collision))


def feq(q, rho, u):
    _, s = one_cell(q)
    s.init_lbm(np.array([[rho], [u[0]], [u[1]], [u[2]]]))
    return s.get_f()[0]


@pytest.mark.parametrize("q", [19, 27])
def test_weights_are_isotropic_to_fourth_order(q):
    w = feq(q, 1.0, (0.0, 0.0, 0.0))
    n_nonzero = int((w > 0).sum())
    assert n_nonzero == q
    assert abs(w.sum() - 1.0) <= 1e-15
    d = np.eye(3)
    m2 = np.einsum("i,ia,ib->ab", w, C, C)
    assert np.abs(m2 - CS2 * d).max() <= 1e-15
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, C, C, C, C)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d))
    assert np.abs(m4 - iso).max() <= 1e-15
    assert np.abs(np.einsum("i,ia->a", w, C)).max() <= 1e-16
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, C, C, C)).max() <= 1e-16


@pytest.mark.parametrize("q", [19, 27])
def test_equilibrium_moments(q):
    rho, u = 1.3, np.array([0.1, -0.05, 0.08])
    f = feq(q, rho, u)
    assert abs(f.sum() - rho) <= 1e-15 * rho
    assert np.abs(C.T @ f - rho * u).max() <= 1e-15
    P = np.einsum("i,ia,ib->ab", f, C, C)
    assert np.abs(P - (rho * CS2 * np.eye(3) + rho * np.outer(u, u))).max() <= 1e-15
    if q == 19:
        corners = np.abs(C).sum(1) == 3
        assert np.all(f[corners] == 0.0)


@pytest.mark.parametrize("q", [19, 27])
def test_homogeneous_relaxation_closed_form_and_conservation(q):
    """one cell, periodic onto itself (transport cancels): f^n = f_eq + (f^0 - f_eq) e^{-n dt/tau}"""
    tau = 0.7
    m, s = one_cell(q, tau)
    rng = np.random.default_rng(q)
    f0 = feq(q, 1.0, (0.05, 0.0, -0.03)) * (1.0 + 0.3 * rng.random(27))
    s.set_f(f0[None, :])
    rho = f0.sum()
    u = (C.T @ f0) / rho
    fe = feq(q, rho, u)
    dt = 0.05
    for n in range(1, 6):
        assert s.step(dt, 1) == 0
        got = s.get_f()[0]
        want = fe + (f0 - fe) * math.exp(-n * dt / tau)
        assert np.abs(got - want).max() <= 1e-14 * np.abs(f0).max()
        assert abs(got.sum() - rho) <= 1e-14 * rho
        assert np.abs(C.T @ got - rho * u).max() <= 1e-14 * rho


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.08, -0.05, 0.03)])
def test_uniform_equilibrium_stationary_on_octree(q, u):
    f = balanced(I.random_forest(3, (2, 2, 2), 2, 0.3))
    m = O.Mesh(f)
    s = O.Solver(m, O.lbm_params(q, 0.6))
    s.init_lbm(np.tile(np.array([[1.1], [u[0]], [u[1]], [u[2]]]), (1, s.n)))
    f0 = s.get_f()
    assert s.step(s.dt_cfl(0.5), 10) == 0
    assert np.abs(s.get_f() - f0).max() <= 1e-14 * np.abs(f0).max()


@pytest.mark.parametrize("q", [19, 27])
def test_periodic_octree_conserves_mass_and_momentum(q):
    f = balanced(I.random_forest(5, (2, 2, 2), 2, 0.3))
    m = O.Mesh(f)
    t = m.tables()
    s = O.Solver(m, O.lbm_params(q, 0.6))
    x = I.leaf_centres(f)[t["input"]]
    prim = np.stack([1 + 0.1 * np.sin(2 * np.pi * x[:, 0]), 0.05 * np.cos(2 * np.pi * x[:, 1]),
                     0.04 * np.sin(2 * np.pi * x[:, 2]), 0 * x[:, 0]])
    s.init_lbm(prim)
    g0 = s.global_sums()
    assert s.step(s.dt_cfl(0.5), 8) == 0
    g1 = s.global_sums()
    assert np.abs(g1[:4] - g0[:4]).max() <= 1e-13 * g0[0]
    fq = s.get_f()
    if q == 19:
        assert np.all(fq[:, np.abs(C).sum(1) == 3] == 0.0)
    assert np.abs(fq - s.get_f()).max() == 0.0


def test_lbm_grid_is_checked():
    m = O.Mesh(I.uniform_forest((1, 1, 1), 1))
    with pytest.raises(RuntimeError):
        O.Solver(m, O.make_params((3, 3, 3), (-1.5,) * 3, (1.5,) * 3, collision=4, lbm_q=15))
    with pytest.raises(RuntimeError):
        O.Solver(m, O.make_params((4, 4, 4), (-2.0,) * 3, (2.0,) * 3, collision=4, lbm_q=19))


def balanced(forest):
    lev, ijk = O.balance(forest)
    return dataclasses.replace(forest, level=lev, ijk=ijk)
