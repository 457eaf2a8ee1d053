"""Pins of the oracle's MUSCL-minmod transport at octree level jumps and at
domain boundaries (reading S12 of eq. 2: normal-direction slope from the
one-sided differences to the face-neighbour values, the mean of the four
leaves across a FINER face, over the distances between cell centres; no slope
in leaves that touch a wall; ghosts carry no slope).

Two independent checks of the same reading:
- a profile linear in x is advected exactly, f* = f - dt xi_x b, in every
  cell whose stencil stays inside the domain: any error in the FINER mean, in
  the face offset h/2 or a centre distance that shrinks a slope breaks it;
- a brute-force MUSCL step written from geometry alone (neighbours from the
  O(n^2) shared-face enumeration, centre distances and sub-face areas from the
  leaf coordinates, not from the per-kind constants), compared cell by cell
  on random data, where minmod picks either side, so a distance too large or
  too small on any kind of face shows.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_00707_amd import inputs as I


def balanced(forest):
    lev, ijk = O.balance(forest)
    return dataclasses.replace(forest, level=lev, ijk=ijk)


def solver_for(forest, nv, lo, hi, **kw):
    m = O.Mesh(forest, kw.pop("solid", None))
    return m, O.Solver(m, O.make_params(nv, lo, hi, **kw))


def vgrid(nv, lo, hi):
    xs = [lo[a] + (np.arange(nv[a]) + 0.5) * (hi[a] - lo[a]) / nv[a] for a in range(3)]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()])


def _jump_forest(seed):
    """4 x 2 x 2 roots, random refinement up to 2 levels, 2:1 balanced, open in x"""
    bc = (I.OUTFLOW,) * 6
    return balanced(I.random_forest(seed, (4, 2, 2), 2, 0.35, bc))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_muscl_linear_profile_exact_across_level_jumps(seed):
    """xi_y = xi_z = 0 and f = a_i + b_i x: with every slope of the stencil
    unlimited (both one-sided differences equal b_i), upwind face values are
    a_i + b_i x_face, so the flux difference over the cell is exact and
    f* = f - dt xi_x b_i in every cell whose own x-faces and upwind cells'
    x-faces are interior."""
    f = _jump_forest(seed)
    nv, lo, hi = (6, 1, 1), (-3.0, -0.5, -0.5), (3.0, 0.5, 0.5)
    m, s = solver_for(f, nv, lo, hi, collision=2, scheme=1)
    t = m.tables()
    h = f.h0 / 2.0 ** t["level"].astype(np.float64)
    x = (t["ijk"][:, 0] + 0.5) * h
    xi = vgrid(nv, lo, hi)[0]
    rng = np.random.default_rng(100 + seed)
    b = rng.uniform(-0.6, 0.6, nv[0])
    b[np.abs(b) < 0.1] = 0.3
    a = 3.0 + rng.random(nv[0])
    f0 = a[None, :] + b[None, :] * x[:, None]
    s.set_f(f0)
    dt = s.dt_cfl(0.5)
    s.transport(dt)
    got = s.get_f()
    ty, nb = t["type"], t["nbr"]
    interior_x = (ty[:, 0] <= O.FACE_FINER) & (ty[:, 1] <= O.FACE_FINER)
    checked = {O.FACE_SAME: 0, O.FACE_COARSER: 0, O.FACE_FINER: 0}
    for c in range(s.n):
        if not interior_x[c]:
            continue
        for v in range(nv[0]):
            up = 0 if xi[v] > 0 else 1          # the upwind x-face
            k = 4 if ty[c, up] == O.FACE_FINER else 1
            ups = nb[c, up, :k]
            if not interior_x[ups].all():
                continue
            want = f0[c, v] - dt * xi[v] * b[v]
            assert abs(got[c, v] - want) <= 1e-14 * abs(f0[c, v]), (c, v, got[c, v], want)
            checked[int(ty[c, up])] += 1
    # the pin covers upwind faces of every kind
    assert all(n > 10 for n in checked.values()), checked


def _brute_muscl_transport(forest, nv, lo, hi, f0, dt, ghost_in, distance_error=None):
    """f* of one forward-Euler MUSCL-minmod step from the leaf geometry alone.
    distance_error = (kind, factor) scales the centre distance over faces of
    that kind (a planted mistake, to show the comparison is sensitive)."""
    order, ty, nb = O.brute_faces(forest)
    lev = forest.level[order].astype(np.float64)
    h = forest.h0 / 2.0 ** lev
    ctr = (forest.ijk[order].astype(np.float64) + 0.5) * h[:, None]
    L = np.array(forest.base, np.float64) * forest.h0
    n = len(order)
    xi = vgrid(nv, lo, hi)

    def nb_list(c, face):
        k = ty[c, face]
        if k == O.FACE_FINER:
            return list(nb[c, face])
        if k in (O.FACE_SAME, O.FACE_COARSER):
            return [nb[c, face, 0]]
        return []

    def minmod(p, q):
        return np.where(p * q <= 0, 0.0, np.where(np.abs(p) < np.abs(q), p, q))

    sig = np.zeros((n, 3, f0.shape[1]))
    for c in range(n):
        for ax in range(3):
            side_val, side_d = [], []
            for side in (0, 1):
                face = 2 * ax + side
                lst = nb_list(c, face)
                if lst:
                    # area-weighted mean value and centre of the face's leaves
                    area = np.array([h[q] ** 2 if h[q] <= h[c] else h[c] ** 2 for q in lst])
                    val = (area[:, None] * f0[lst]).sum(0) / area.sum()
                    cx = (area * ctr[lst, ax]).sum() / area.sum()
                    d = (ctr[c, ax] - cx) % L[ax] if side == 0 else (cx - ctr[c, ax]) % L[ax]
                    if distance_error is not None and ty[c, face] == distance_error[0]:
                        d *= distance_error[1]
                else:
                    kind = ty[c, face]
                    val = ghost_in if kind == O.FACE_INFLOW else f0[c]
                    d = h[c]                      # a mirror ghost of the cell's size
                side_val.append(val)
                side_d.append(d)
            sig[c, ax] = minmod((f0[c] - side_val[0]) / side_d[0], (side_val[1] - f0[c]) / side_d[1])

    fn = f0.copy()
    for c in range(n):
        acc = np.zeros(f0.shape[1])
        for face in range(6):
            ax, sgn = face // 2, (1.0 if face % 2 else -1.0)
            xn = sgn * xi[ax]
            out = xn > 0
            own_face = f0[c] + sgn * 0.5 * h[c] * sig[c, ax]
            lst = nb_list(c, face)
            if lst:
                for q in lst:
                    A = min(h[q], h[c]) ** 2
                    nb_face = f0[q] - sgn * 0.5 * h[q] * sig[q, ax]
                    acc += A * xn * np.where(out, own_face, nb_face)
            else:
                ghost = ghost_in if ty[c, face] == O.FACE_INFLOW else f0[c]
                acc += h[c] ** 2 * xn * np.where(out, own_face, ghost)
        fn[c] = f0[c] - dt / h[c] ** 3 * acc
    return fn


@pytest.mark.parametrize("seed,base,levels,open_", [(0, (2, 2, 2), 3, False), (1, (2, 2, 2), 3, False),
                                                     (2, (3, 2, 2), 2, True), (3, (2, 2, 2), 3, True)])
def test_muscl_step_equals_geometric_bruteforce(seed, base, levels, open_):
    bc = (I.INFLOW,) + (I.OUTFLOW,) * 5 if open_ else (I.PERIODIC,) * 6
    f = balanced(I.random_forest(seed, base, levels, 0.25, bc))
    nv, lo, hi = (4, 4, 4), (-3.0,) * 3, (3.0,) * 3
    prim_in = (1.1, 0.7, -0.2, 0.1, 0.9)
    m, s = solver_for(f, nv, lo, hi, collision=2, scheme=1, inflow=prim_in)
    t = m.tables()
    kinds = set(np.unique(t["type"]).tolist())
    assert {O.FACE_COARSER, O.FACE_FINER} <= kinds
    rng = np.random.default_rng(50 + seed)
    f0 = 1.0 + rng.random((s.n, s.nv))
    s.set_f(f0)
    dt = s.dt_cfl(0.5)
    s.transport(dt)
    got = s.get_f()
    ghost = O.cell_maxwellian(nv, lo, hi, prim_in)
    want = _brute_muscl_transport(f, nv, lo, hi, f0, dt, ghost)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(f0))
    # the transport did move something at every kind of face
    assert np.max(np.abs(got - f0)) > 1e-3


@pytest.mark.parametrize("kind,factor", [(O.FACE_COARSER, 2.0 / 3.0), (O.FACE_COARSER, 4.0 / 3.0),
                                         (O.FACE_FINER, 4.0 / 3.0), (O.FACE_FINER, 2.0 / 3.0),
                                         (O.FACE_SAME, 1.5)])
def test_bruteforce_muscl_sees_a_wrong_centre_distance(kind, factor):
    """The comparison above is not vacuous: the brute force with one centre
    distance rule changed (e.g. h instead of 3h/2 across a COARSER face, h
    instead of 3h/4 across a FINER one) disagrees with the oracle."""
    f = balanced(I.random_forest(1, (2, 2, 2), 3, 0.25, (I.PERIODIC,) * 6))
    nv, lo, hi = (4, 4, 4), (-3.0,) * 3, (3.0,) * 3
    m, s = solver_for(f, nv, lo, hi, collision=2, scheme=1)
    rng = np.random.default_rng(51)
    f0 = 1.0 + rng.random((s.n, s.nv))
    s.set_f(f0)
    dt = s.dt_cfl(0.5)
    s.transport(dt)
    got = s.get_f()
    right = _brute_muscl_transport(f, nv, lo, hi, f0, dt, None)
    wrong = _brute_muscl_transport(f, nv, lo, hi, f0, dt, None, distance_error=(kind, factor))
    assert np.max(np.abs(got - right)) <= 1e-13 * np.max(np.abs(f0))
    assert np.max(np.abs(got - wrong)) > 1e-6 * np.max(np.abs(f0))


@pytest.mark.parametrize("scheme", [0, 1])
def test_free_stream_inflow_outflow_stationary_both_schemes(scheme):
    nv, lo, hi = (8, 8, 8), (-6.0,) * 3, (6.0,) * 3
    bc = (I.INFLOW,) + (I.OUTFLOW,) * 5
    f = balanced(dataclasses.replace(I.random_forest(4, (2, 2, 2), 2, 0.3), bc=bc))
    prim_in = (1.0, 1.5, 0.0, 0.0, 1.0)
    m, s = solver_for(f, nv, lo, hi, tau_or_kn=0.1, inflow=prim_in, scheme=scheme)
    s.init_maxwellian(np.tile(np.array(prim_in)[:, None], (1, s.n)))
    f0 = s.get_f()
    assert s.step(s.dt_cfl(0.5), 10) == 0
    assert np.max(np.abs(s.get_f() - f0)) <= 1e-14 * np.max(f0)


def test_muscl_closed_box_diffuse_wall_mass_tight():
    """Walls pass no mass only if the value leaving through a wall face is the
    one the wall density was computed from: MUSCL must carry no slope in
    leaves that touch a wall (reading S12).  Gas at rest at T_w stays put."""
    nv, lo, hi = (8, 8, 8), (-4.5,) * 3, (4.5,) * 3
    f = balanced(dataclasses.replace(I.random_forest(5, (2, 2, 2), 2, 0.3), bc=(I.WALL,) * 6))
    m, s = solver_for(f, nv, lo, hi, tau_or_kn=0.1, t_wall=0.8, scheme=1)
    s.init_maxwellian(np.tile(np.array([[0.9], [0.0], [0.0], [0.0], [0.8]]), (1, s.n)))
    f0 = s.get_f()
    assert s.step(s.dt_cfl(0.5), 10) == 0
    assert np.max(np.abs(s.get_f() - f0)) <= 1e-14 * np.max(f0)
    t = m.tables()
    h = f.h0 / 2.0 ** t["level"]
    x = (t["ijk"] + 0.5) * h[:, None]
    prim = np.stack([1 + 0.3 * np.sin(2 * np.pi * x[:, 0]), 0.2 * np.cos(2 * np.pi * x[:, 1]),
                     0 * x[:, 0], 0 * x[:, 0], 1 + 0.2 * x[:, 2]])
    s.init_maxwellian(prim)
    g0 = s.global_sums()
    assert s.step(s.dt_cfl(0.5), 10) == 0
    g1 = s.global_sums()
    assert abs(g1[0] - g0[0]) <= 1e-13 * g0[0]
    assert abs(g1[4] - g0[4]) > 1e-6 * g0[4]


def test_muscl_wall_box_solid_sphere_mass_tight():
    """The same with fluid-solid WALL faces of a staircase sphere inside a
    periodic box: mass is conserved to rounding under MUSCL."""
    f = I.sphere_refinement(base=(4, 4, 4), levels=2, radius=0.3)
    f = balanced(dataclasses.replace(f, bc=(I.PERIODIC,) * 6))
    sol = I.solid_flags(f, (0.5, 0.5, 0.5), 0.3, 2)
    nv, lo, hi = (6, 6, 6), (-4.5,) * 3, (4.5,) * 3
    m, s = solver_for(f, nv, lo, hi, tau_or_kn=0.1, t_wall=1.2, scheme=1, solid=sol)
    t = m.tables()
    assert (t["type"] == O.FACE_WALL).sum() > 0
    h = f.h0 / 2.0 ** t["level"]
    x = (t["ijk"] + 0.5) * h[:, None]
    prim = np.stack([1 + 0.2 * np.sin(2 * np.pi * x[:, 0]), 0.3 + 0 * x[:, 0], 0 * x[:, 0], 0 * x[:, 0],
                     1 + 0.1 * np.cos(2 * np.pi * x[:, 2])])
    s.init_maxwellian(prim)
    g0 = s.global_sums()
    assert s.step(s.dt_cfl(0.5), 8) == 0
    g1 = s.global_sums()
    assert abs(g1[0] - g0[0]) <= 1e-13 * g0[0]
