"""Pins of the oracle's Boltzmann collision integral on Korobov lattice nodes
(section 3.2, eqs. 3-6) against what the mathematics fixes: Korobov's
optimal generator by brute force, the tables rebuilt independently from
their definition, uniform partner marginals of a rank-1 lattice, the closed-
form hard-sphere collision frequency of a Maxwellian, exact conservation of
mass, momentum and energy after the correction of eq. 6, the Maxwellian as
a fixed point up to a quadrature error that falls with the lattice size,
the scaling of the loss (linear) and gain (quadratic) terms, and relaxation
of a two-beam distribution toward equilibrium."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import oracle as O
from paper_1503_00707_amd import inputs as I

NV, LO, HI = (8, 8, 8), (-4.5,) * 3, (4.5,) * 3


def grid(nv, lo, hi):
    xs = [lo[a] + (np.arange(nv[a]) + 0.5) * (hi[a] - lo[a]) / nv[a] for a in range(3)]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    w = np.prod([(hi[a] - lo[a]) / nv[a] for a in range(3)])
    return X.ravel(), Y.ravel(), Z.ravel(), w


def test_generator_is_korobov_optimal_by_brute_force():
    """the first a in 2..p-1 minimising P_2 = -1 + mean_k prod_d (1 + 2 pi^2 B_2({k a^d / p}))
    (a, -a, 1/a, -1/a mod p tie exactly: the same lattice up to coordinate order and sign)"""
    for p in (31, 101, 127):
        best, best_v = None, None
        k = np.arange(p, dtype=np.int64)
        for a in range(2, p):
            prod = np.ones(p)
            z = k.copy()
            for d in range(5):
                x = z / p
                prod *= 1 + 2 * math.pi ** 2 * (x * x - x + 1 / 6)
                z = (z * a) % p
            v = -1 + prod.mean()
            if best_v is None or v < best_v - 1e-9 * abs(best_v):
                best, best_v = a, v
        assert O.korobov_generator(p) == best
    assert O.korobov_generator(100) == -1  # not prime


def _tables_from_definition(nv, lo, hi, p, a):
    """the tables written out from their definition, one trial at a time"""
    d = [(hi[b] - lo[b]) / nv[b] for b in range(3)]
    xs = [[lo[b] + (q + 0.5) * d[b] for q in range(nv[b])] for b in range(3)]
    vbox = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2])
    c = [((2654435761 % p) * (e + 1)) % p for e in range(5)]
    n = nv[0] * nv[1] * nv[2]
    J, L, M = (np.zeros((n, p), np.int64) for _ in range(3))
    W = np.zeros((n, p))

    def node(b, v):
        t = math.floor((v - lo[b]) / d[b])
        return t if 0 <= t < nv[b] else -1

    for i in range(n):
        ix, iy, iz = i // (nv[1] * nv[2]), (i // nv[2]) % nv[1], i % nv[2]
        xi = (xs[0][ix], xs[1][iy], xs[2][iz])
        for k in range(p):
            q = [(k * pow(a, e, p) + (i + 1) * c[e]) % p for e in range(5)]
            jb = [((2 * q[b] + 1) * nv[b]) // (2 * p) for b in range(3)]
            xst = (xs[0][jb[0]], xs[1][jb[1]], xs[2][jb[2]])
            g = [xst[b] - xi[b] for b in range(3)]
            gg = math.sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2])
            ct = 1.0 - 2.0 * ((q[3] + 0.5) / p)
            st = math.sqrt(max(0.0, 1.0 - ct * ct))
            ph = 2.0 * math.pi * ((q[4] + 0.5) / p)
            nn = (st * math.cos(ph), st * math.sin(ph), ct)
            l1 = [node(b, 0.5 * (xi[b] + xst[b]) + 0.5 * gg * nn[b]) for b in range(3)]
            l2 = [node(b, 0.5 * (xi[b] + xst[b]) - 0.5 * gg * nn[b]) for b in range(3)]
            ok = min(l1) >= 0 and min(l2) >= 0
            J[i, k] = (jb[0] * nv[1] + jb[1]) * nv[2] + jb[2]
            L[i, k] = (l1[0] * nv[1] + l1[1]) * nv[2] + l1[2] if ok else -1
            M[i, k] = (l2[0] * nv[1] + l2[1]) * nv[2] + l2[2] if ok else -1
            W[i, k] = vbox * gg / p
    return J, L, M, W


@pytest.mark.parametrize("nv,p", [((4, 4, 4), 31), ((4, 6, 2), 61)])
def test_tables_equal_their_definition(nv, p):
    lo, hi = (-3.0, -2.5, -2.0), (3.0, 2.5, 2.0)
    a = O.korobov_generator(p)
    j, l, m, W = O.korobov_tables(nv, lo, hi, p, a)
    J, L, M, Wd = _tables_from_definition(nv, lo, hi, p, a)
    assert np.array_equal(j, J) and np.array_equal(l, L) and np.array_equal(m, M)
    assert np.abs(W - Wd).max() <= 1e-15 * Wd.max()
    assert (l < 0).any() and (l >= 0).mean() > 0.3    # some trials leave the grid, most stay


def test_partner_marginals_are_uniform():
    """a rank-1 lattice visits every value of each coordinate once, so each
    axis index of the partner node is hit p/N times, to within one"""
    p = 1021
    j, _, _, _ = O.korobov_tables(NV, LO, HI, p, O.korobov_generator(p))
    for i in (0, 137, 511):
        jb = [j[i] // 64, (j[i] // 8) % 8, j[i] % 8]
        for b in range(3):
            cnt = np.bincount(jb[b], minlength=8)
            assert cnt.max() - cnt.min() <= 1 and cnt.sum() == p


def test_collision_frequency_of_a_maxwellian_matches_the_closed_form():
    """B of eq. 4 for f = M(rho, u, T) is the hard-sphere collision frequency
    nu = rho sqrt(2T) (exp(-s^2)/sqrt(pi) + (s + 1/(2s)) erf(s)), s = |xi - u| / sqrt(2T),
    up to the velocity grid's and the lattice rule's errors; the full
    discrete sum sum_j w |xi_i - xi_j| f_j sits between the two"""
    nv, lo, hi = (16, 16, 16), (-6.0,) * 3, (6.0,) * 3
    X, Y, Z, w = grid(nv, lo, hi)
    rho, u, T = 1.3, np.array([0.4, -0.3, 0.2]), 0.9
    f = O.cell_maxwellian(nv, lo, hi, (rho, *u, T))
    s = np.sqrt((X - u[0]) ** 2 + (Y - u[1]) ** 2 + (Z - u[2]) ** 2) / math.sqrt(2 * T)
    nu = rho * math.sqrt(2 * T) * (np.exp(-s ** 2) / math.sqrt(math.pi) + (s + 1 / (2 * s)) * erf(s))
    G = np.sqrt((X[:, None] - X[None, :]) ** 2 + (Y[:, None] - Y[None, :]) ** 2 + (Z[:, None] - Z[None, :]) ** 2)
    Bd = (G * w) @ f
    assert np.abs(Bd - nu).max() <= 5e-3 * nu.max()
    errs, rate = [], []
    for p in (1021, 4093):
        _, B, _ = O.korobov_cell(nv, lo, hi, p, O.korobov_generator(p), f)
        errs.append(np.abs(B - Bd).max() / Bd.max())
        # the total collision rate sum_i w f_i B_i averages the lattice error out
        rate.append(abs(w * (f @ B) - w * (f @ Bd)) / (w * (f @ Bd)))
    assert errs[1] < errs[0] and errs[1] <= 0.1, errs
    assert max(rate) <= 1e-2, rate


@pytest.mark.parametrize("kind", ["maxwellian", "random", "two_beam"])
def test_corrected_integral_conserves_mass_momentum_energy(kind):
    X, Y, Z, w = grid(NV, LO, HI)
    if kind == "maxwellian":
        f = O.cell_maxwellian(NV, LO, HI, (0.8, 0.5, -0.4, 0.2, 1.4))
    elif kind == "random":
        f = np.random.default_rng(3).random(X.size) * np.exp(-(X * X + Y * Y + Z * Z) / 6)
    else:
        f = np.exp(-((X - 1.5) ** 2 + Y ** 2 + Z ** 2) / 1.0) + np.exp(-((X + 1.5) ** 2 + Y ** 2 + Z ** 2) / 1.0)
    p = 1021
    Ival, B, C = O.korobov_cell(NV, LO, HI, p, O.korobov_generator(p), f)
    psi = np.stack([np.ones_like(X), X, Y, Z, X * X + Y * Y + Z * Z])
    scale = np.abs(psi) @ np.abs(f * B) * w
    assert np.all(np.abs(psi @ Ival * w) <= 1e-13 * scale)
    # the uncorrected integral C - f B does not conserve by itself (eq. 6 is needed)
    raw = psi @ (C - f * B) * w
    assert np.abs(raw).max() > 1e-6 * scale.max()


def test_maxwellian_is_a_fixed_point_up_to_the_quadrature_error():
    f = O.cell_maxwellian(NV, LO, HI, (1.0, 0.3, -0.2, 0.1, 1.0))
    res = []
    for p in (127, 1021, 4093):
        Ival, B, _ = O.korobov_cell(NV, LO, HI, p, O.korobov_generator(p), f)
        res.append(np.abs(Ival).max() / np.max(f * B))
    assert res[2] < res[1] < res[0] and res[2] <= 0.05, res


def test_loss_is_linear_and_gain_quadratic_in_f():
    X, Y, Z, w = grid(NV, LO, HI)
    f = np.random.default_rng(5).random(X.size)
    p = 251
    a = O.korobov_generator(p)
    _, B1, C1 = O.korobov_cell(NV, LO, HI, p, a, f)
    _, B3, C3 = O.korobov_cell(NV, LO, HI, p, a, 3.0 * f)
    assert np.abs(B3 - 3 * B1).max() <= 1e-14 * np.abs(B3).max()
    assert np.abs(C3 - 9 * C1).max() <= 1e-14 * np.abs(C3).max()


def test_two_beams_relax_toward_equilibrium():
    """homogeneous gas of unit density, f' = f + dt/Kn I(f) with dt/Kn small
    against 1/max B: moments stay; the distance to the Maxwellian of those
    moments falls tenfold, down to the discrete operator's own equilibrium
    (which differs from the Maxwellian by the quadrature error)"""
    X, Y, Z, w = grid(NV, LO, HI)
    f = np.exp(-((X - 1.5) ** 2 + Y ** 2 + Z ** 2) / 0.8) + np.exp(-((X + 1.5) ** 2 + Y ** 2 + Z ** 2) / 0.8)
    f = f / O.cell_moments(NV, LO, HI, f)[0]
    p = 1021
    a = O.korobov_generator(p)
    m0 = O.cell_moments(NV, LO, HI, f)
    rho = m0[0]
    u = m0[1:4] / rho
    T = (2 * m0[4] / rho - u @ u) / 3
    Mt = O.cell_maxwellian(NV, LO, HI, (rho, *u, T))
    dist = [np.abs(f - Mt).max()]
    dt_kn = 0.05
    for _ in range(60):
        Ival, B, _ = O.korobov_cell(NV, LO, HI, p, a, f)
        assert dt_kn * B.max() < 0.5
        f = f + dt_kn * Ival
        dist.append(np.abs(f - Mt).max())
        m = O.cell_moments(NV, LO, HI, f)
        # each step conserves to the rounding of the 5x5 solve (raw basis of eq. 6)
        assert np.abs(m - m0).max() <= 1e-12 * np.abs(m0).max()
    assert all(dist[k + 6] < dist[k] for k in range(0, 36, 6))
    assert dist[36] < 0.1 * dist[0] and max(dist[36:]) < 0.1 * dist[0]


def test_solver_korobov_collision_conserves_on_an_octree():
    """the solver's step with the Korobov collision (transport, then
    f' = f* + dt/Kn I(f*)): global mass, momentum and energy conserved on a
    periodic octree; a uniform state stays uniform"""
    import dataclasses
    lev, ijk = O.balance(I.random_forest(3, (2, 2, 2), 2, 0.3))
    f = dataclasses.replace(I.random_forest(3, (2, 2, 2), 2, 0.3), level=lev, ijk=ijk)
    m = O.Mesh(f)
    t = m.tables()
    s = O.Solver(m, O.make_params(NV, LO, HI, collision=3, tau_or_kn=0.5, korobov_p=127))
    x = I.leaf_centres(f)[t["input"]]
    s.init_maxwellian(I.fields("sines", x, seed=4))
    g0 = s.global_sums()
    dt = s.dt_cfl(0.5)
    assert s.step(dt, 4) == 0
    g1 = s.global_sums()
    sc = np.array([g0[0]] * 4 + [g0[4]])
    assert np.all(np.abs(g1 - g0) <= 1e-13 * sc)
    u = O.Solver(m, O.make_params(NV, LO, HI, collision=3, tau_or_kn=0.5, korobov_p=127))
    u.init_maxwellian(np.tile(np.array([[1.0], [0.2], [0.0], [-0.1], [1.1]]), (1, u.n)))
    u.step(dt, 2)
    fu = u.get_f()
    assert np.abs(fu - fu[0][None, :]).max() <= 1e-14 * np.abs(fu).max()
