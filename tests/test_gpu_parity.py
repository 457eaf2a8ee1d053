"""Parity of the HIP path (called through the C interface) with the FP64
oracle on the same seeded inputs: FP64 within 1e-12 relative, FP32 storage
with FP64 sums within 2e-5 relative L-inf on the moments after 20 steps."""
import dataclasses

import numpy as np
import pytest

from paper_1503_00707_amd import dvm as D
from paper_1503_00707_amd import inputs as I
from tests.gpu_common import Case, balanced, gpu_run, gpu_solver, moment_errors, oracle_run, prim_for

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-5


def _uniform16_v8():
    w = I.workload("uniform16_v8_fp64")
    return Case(w.forest, 8, 4.5, tau=0.1, fields="sine_rho", field_args={"a": 0.1})


def sums_errors(g, ref, mom_ref):
    """global FP64 sums sum_c V_c (rho, rho u, E): per-component error over
    (total mass, total mass sqrt(max T) for the momenta, total energy)"""
    rho = mom_ref[0]
    u = mom_ref[1:4] / rho
    T = (2 * mom_ref[4] / rho - (u * u).sum(0)) / 3
    su = abs(ref[0]) * float(np.sqrt(T.max()))
    scale = np.array([abs(ref[0]), su, su, su, abs(ref[4])])
    return np.abs(np.asarray(g) - ref) / scale


def _compare(case, steps, precision, tol, f_tol=None):
    """moments (and the step's own moments buffer), the global sums reported
    by dvm_check and f against the oracle.  FP32 storage: f within 2e-5 of
    max |f| unless f_tol says otherwise."""
    o = oracle_run(case, steps)
    g = gpu_run(case, steps, precision)
    assert o["rc"] == 0 and g["rc"] == 0
    assert g["dt"] == pytest.approx(o["dt"], rel=1e-15)
    err = moment_errors(g["mom"], o["mom"])
    print("moment errors", err)
    assert np.all(err <= tol), err
    # the moments written by the step (post-transport, conserved by the collision)
    err_step = moment_errors(g["mom_step"], o["mom"])
    assert np.all(err_step <= max(tol, 1e-12)), err_step
    # global conservation sums (dvm_check) against the oracle's
    es = sums_errors(g["sums"], o["sums"], o["mom"])
    print("global sums errors", es)
    assert np.all(es <= tol), es
    if f_tol is None and precision == D.PREC_FP32:
        f_tol = FP32_TOL
    if f_tol is not None:
        ef = np.abs(g["f"] - o["f"]).max() / np.abs(o["f"]).max()
        print("f error", ef)
        assert ef <= f_tol
    return o, g


def test_uniform16_v8_fp64_20_steps():
    _compare(_uniform16_v8(), 20, D.PREC_FP64, FP64_TOL, f_tol=FP64_TOL)


def test_uniform16_v8_fp32_20_steps():
    _compare(_uniform16_v8(), 20, D.PREC_FP32, FP32_TOL)


@pytest.mark.parametrize("seed", [0, 1])
def test_octree_periodic_fp64(seed):
    f = balanced(I.random_forest(seed, (2, 2, 2), 3, 0.2))
    case = Case(f, 8, 4.5, tau=0.05, fields="sines", field_args={"seed": 100 + seed})
    _compare(case, 10, D.PREC_FP64, FP64_TOL, f_tol=FP64_TOL)


@pytest.mark.parametrize("coll", [I.COLL_EULER, I.COLL_OFF])
def test_octree_collision_modes_fp64(coll):
    f = balanced(I.random_forest(2, (2, 2, 2), 2, 0.3))
    case = Case(f, 8, 4.5, tau=0.2, collision=coll, fields="sines", field_args={"seed": 7})
    _compare(case, 6, D.PREC_FP64, FP64_TOL, f_tol=FP64_TOL)


def test_octree_inflow_outflow_wall_fp64():
    bc = (I.INFLOW, I.OUTFLOW, I.WALL, I.WALL, I.OUTFLOW, I.OUTFLOW)
    f = balanced(I.random_forest(3, (2, 2, 2), 3, 0.2, bc))
    case = Case(f, 8, 6.0, tau_mode=I.TAU_HS, tau=0.05, inflow=(1.0, 1.3, 0.1, 0.0, 1.1), t_wall=0.9,
                fields="sines", field_args={"seed": 9})
    _compare(case, 8, D.PREC_FP64, FP64_TOL, f_tol=FP64_TOL)


def test_sphere_solid_inflow_fp64():
    f = balanced(I.sphere_refinement(base=(8, 8, 8), levels=2, radius=0.2))
    sol = I.solid_flags(f, (0.5, 0.5, 0.5), 0.2, 2)
    u_in = 2.0 * (5.0 / 3.0) ** 0.5
    case = Case(f, 8, 6.0, tau_mode=I.TAU_HS, tau=0.05, inflow=(1.0, u_in, 0.0, 0.0, 1.0), solid=sol,
                fields="uniform", field_args={"rho": 1.0, "u": (u_in, 0.0, 0.0), "T": 1.0})
    _compare(case, 8, D.PREC_FP64, FP64_TOL, f_tol=FP64_TOL)


@pytest.mark.parametrize("nv,vmax", [(12, 6.0), (16, 6.0), (24, 6.0)])
def test_octree_sod_hard_sphere(nv, vmax):
    """the paper-scale construction (roots refined once at random, Sod-like jump,
    tau from Kn) on 4^3 roots: FP64 to 1e-12, FP32 to 2e-5 after 20 steps"""
    f = I.random_root_refinement((4, 4, 4), 0.4, 3)
    case = Case(f, nv, vmax, tau_mode=I.TAU_HS, tau=0.01, fields="sod_x")
    o, g = _compare(case, 20, D.PREC_FP32, FP32_TOL)
    g64 = gpu_run(case, 20, D.PREC_FP64)
    err = moment_errors(g64["mom"], o["mom"])
    assert np.all(err <= FP64_TOL), err
    ef = np.abs(g64["f"] - o["f"]).max() / np.abs(o["f"]).max()
    assert ef <= FP64_TOL


def test_stationary_maxwellian_and_conservation():
    import torch
    f = balanced(I.random_forest(4, (2, 2, 2), 3, 0.2))
    case = Case(f, 8, 4.5, fields="uniform", field_args={"rho": 1.1, "u": (0.2, -0.1, 0.3), "T": 0.9})
    dm, s = gpu_solver(case, D.PREC_FP64)
    f0 = s.f_canonical().cpu().numpy()
    s.step(20, cfl=0.5)
    f1 = s.f_canonical().cpu().numpy()
    assert np.abs(f1 - f0).max() <= 1e-14 * np.abs(f0).max()
    # a non-uniform state on a periodic octree: global sums conserved
    case2 = Case(f, 8, 4.5, tau=0.05, fields="sines", field_args={"seed": 3})
    dm, s = gpu_solver(case2, D.PREC_FP64)
    rc, g0, _, _ = s.check()
    s.step(10, cfl=0.5)
    rc, g1, bad, n = s.check()
    assert rc == 0 and not bad and n == 10
    assert np.all(np.abs(g1 - g0) <= 1e-13 * np.abs(g0).max())
    torch.cuda.synchronize()


def test_deterministic_bitwise():
    f = balanced(I.random_forest(5, (2, 2, 2), 3, 0.2))
    case = Case(f, 16, 6.0, tau_mode=I.TAU_HS, tau=0.02, fields="sines", field_args={"seed": 5})
    a = gpu_run(case, 5, D.PREC_FP32)
    b = gpu_run(case, 5, D.PREC_FP32)
    assert np.array_equal(a["f"], b["f"])
    assert np.array_equal(a["mom"], b["mom"])


def test_canonical_roundtrip_and_nonphysical_flag():
    import torch
    f = I.uniform_forest((1, 1, 1), 2)
    case = Case(f, 8, 4.5, fields="uniform")
    dm, s = gpu_solver(case, D.PREC_FP32)
    rng = np.random.default_rng(0)
    x = rng.random((s.n, s.nv)).astype(np.float32)
    s.set_f_canonical(x)
    back = s.f_canonical().cpu().numpy()
    assert np.array_equal(back, x)
    x[5] = -1.0
    s.set_f_canonical(x)
    s.step(1, cfl=0.5)
    rc, sums, bad, n = s.check()
    assert rc == D.ERR_NONPHYSICAL and bad
    torch.cuda.synchronize()


# --- MUSCL-minmod (the oracle's reading of the reconstruction) -------------

@pytest.mark.parametrize("seed", [0, 1])
def test_muscl_octree_periodic_fp64(seed):
    f = balanced(I.random_forest(10 + seed, (2, 2, 2), 3, 0.25))
    case = Case(f, 8, 4.5, scheme=I.SCHEME_MUSCL, tau=0.05, fields="sines", field_args={"seed": 40 + seed})
    _compare(case, 10, D.PREC_FP64, FP64_TOL, f_tol=FP64_TOL)


def test_muscl_inflow_outflow_wall_fp64():
    bc = (I.INFLOW, I.OUTFLOW, I.WALL, I.WALL, I.PERIODIC, I.PERIODIC)
    f = balanced(I.random_forest(12, (2, 2, 2), 3, 0.2, bc))
    case = Case(f, 8, 6.0, scheme=I.SCHEME_MUSCL, tau_mode=I.TAU_HS, tau=0.05, inflow=(1.0, 1.3, 0.1, 0.0, 1.1),
                t_wall=0.9, fields="sines", field_args={"seed": 19})
    _compare(case, 8, D.PREC_FP64, FP64_TOL, f_tol=FP64_TOL)


def test_muscl_sphere_mach2_fp64_and_fp32():
    """the sphere construction (inflow, outflow, staircase diffuse wall) on
    8^3 roots with 12^3 velocities: FP64 to 1e-12, FP32 to 2e-5 on moments"""
    f = balanced(I.sphere_refinement(base=(8, 8, 8), levels=2, radius=0.2))
    sol = I.solid_flags(f, (0.5, 0.5, 0.5), 0.2, 2)
    u_in = 2.0 * (5.0 / 3.0) ** 0.5
    case = Case(f, 12, 6.0, scheme=I.SCHEME_MUSCL, tau_mode=I.TAU_HS, tau=0.05, inflow=(1.0, u_in, 0.0, 0.0, 1.0),
                solid=sol, fields="uniform", field_args={"rho": 1.0, "u": (u_in, 0.0, 0.0), "T": 1.0})
    o, g = _compare(case, 20, D.PREC_FP32, FP32_TOL)
    g64 = gpu_run(case, 20, D.PREC_FP64)
    assert np.all(moment_errors(g64["mom"], o["mom"]) <= FP64_TOL)
    assert np.abs(g64["f"] - o["f"]).max() <= FP64_TOL * np.abs(o["f"]).max()


def test_muscl_sod_24_fp32():
    f = I.random_root_refinement((4, 4, 4), 0.4, 3)
    case = Case(f, 24, 6.0, scheme=I.SCHEME_MUSCL, tau_mode=I.TAU_HS, tau=0.01, fields="sod_x")
    _compare(case, 20, D.PREC_FP32, FP32_TOL)


@pytest.mark.parametrize("precision", [D.PREC_FP64, D.PREC_FP32])
@pytest.mark.parametrize("irr", [(0, 0), (576, 0)])
def test_split_launches_equal_single_launch_bitwise(precision, irr):
    """cells without FINER or WALL faces stepped by the reduced kernel and the
    rest by a second launch (any shape) give the single launch's step bitwise,
    on a mesh with level jumps, inflow, outflow and a wall; the split state
    also matches the oracle"""
    bc = (I.INFLOW, I.OUTFLOW, I.WALL, I.OUTFLOW, I.PERIODIC, I.PERIODIC)
    f = balanced(I.random_forest(9, (2, 2, 2), 3, 0.25, bc))
    case = Case(f, 24, 6.0, tau_mode=I.TAU_HS, tau=0.02, inflow=(1.0, 0.9, 0.0, 0.0, 1.0), t_wall=1.1,
                fields="sines", field_args={"seed": 5})
    out = []
    for split in (1, 0):
        dm, s = gpu_solver(case, precision)
        s.split(split, *irr)
        s.step(3, cfl=case.cfl)
        out.append((s.f_canonical().double().cpu().numpy(), s.moments().cpu().numpy(), s.check()[0]))
    assert out[0][2] == 0 and out[1][2] == 0
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    o = oracle_run(case, 3)
    err = moment_errors(out[0][1], o["mom"])
    assert np.all(err <= (FP64_TOL if precision == D.PREC_FP64 else FP32_TOL)), err


# --- degenerate and edge cases -------------------------------------------

@pytest.mark.parametrize("nv", [4, 8])
@pytest.mark.parametrize("scheme", [I.SCHEME_UPWIND1, I.SCHEME_MUSCL])
@pytest.mark.parametrize("precision", [D.PREC_FP64, D.PREC_FP32])
def test_single_cell_periodic_domain(nv, scheme, precision):
    """One leaf whose six faces wrap onto itself (the smallest mesh), from a
    non-Maxwellian state: the transport of eq. 2 cancels exactly and the step
    is the BGK relaxation alone; the smallest velocity grid (4^3) included."""
    import torch
    from oracle import oracle as O
    f = I.uniform_forest((1, 1, 1), 0)
    case = Case(f, nv, 3.0, scheme=scheme, tau=0.05, fields="uniform")
    rng = np.random.default_rng(nv + 10 * scheme)
    x = 0.05 + rng.random((1, nv ** 3))
    om = O.Mesh(f)
    op = O.make_params((nv,) * 3, (-3.0,) * 3, (3.0,) * 3, scheme=scheme, tau_or_kn=0.05)
    os_ = O.Solver(om, op)
    os_.set_f(x)
    dt = os_.dt_cfl(0.5)
    assert os_.step(dt, 4) == 0
    dm, s = gpu_solver(case, precision)
    s.set_f_canonical(x)
    s.step(4, dt=dt)
    torch.cuda.synchronize()
    fo, fg = os_.get_f(), s.f_canonical().double().cpu().numpy()
    xf = x.astype(np.float32).astype(np.float64) if precision == D.PREC_FP32 else x
    tol = FP64_TOL if precision == D.PREC_FP64 else 1e-5
    assert np.abs(fg - fo).max() <= tol * np.abs(fo).max()
    err = moment_errors(s.moments().cpu().numpy(), os_.moments())
    assert np.all(err <= (FP64_TOL if precision == D.PREC_FP64 else FP32_TOL)), err
    # the relaxation moves f toward the Maxwellian, it does not leave it
    assert np.abs(fg - xf).max() > 1e-3
    rc, _, bad, n = s.check()
    assert rc == 0 and not bad and n == 4


@pytest.mark.parametrize("scheme", [I.SCHEME_UPWIND1, I.SCHEME_MUSCL])
def test_smallest_velocity_grid_octree_open_and_wall_fp64(scheme):
    """4^3 velocities (one node per octant axis) on an octree with inflow,
    outflow, wall and periodic faces"""
    bc = (I.INFLOW, I.OUTFLOW, I.WALL, I.OUTFLOW, I.PERIODIC, I.PERIODIC)
    f = balanced(I.random_forest(11, (2, 2, 2), 3, 0.25, bc))
    case = Case(f, 4, 3.5, scheme=scheme, tau=0.04, inflow=(1.0, 0.6, 0.0, 0.1, 1.0), t_wall=1.3,
                fields="sines", field_args={"seed": 44})
    _compare(case, 8, D.PREC_FP64, FP64_TOL, f_tol=FP64_TOL)


@pytest.mark.parametrize("scheme", [I.SCHEME_UPWIND1, I.SCHEME_MUSCL])
def test_xcd_grouping_is_bitwise_neutral_with_ragged_tail(scheme):
    """The XCD-aware order of the workgroups (step kernel, and the MUSCL
    face-value kernel) is a bijection of the cells, with the cells past the
    last whole round of groups left in place; every cell's arithmetic is the
    same whichever order runs it."""
    import torch
    f = balanced(I.random_forest(12, (8, 8, 8), 2, 0.3))  # 6,791 cells
    case = Case(f, 24, 6.0, scheme=scheme, tau_mode=I.TAU_HS, tau=0.02, fields="sines", field_args={"seed": 12})
    dm, s = gpu_solver(case, D.PREC_FP32)
    n = s.n
    assert n > 8 * 512 and n % (8 * 64) != 0 and n % (8 * 512) != 0
    dt = s.dt(case.cfl)
    prim = prim_for(case, dm.tables()["input"])
    ref = None
    for g in (1, 8, 64, 512):
        s.set_shape(192, 31, g, 1)
        s.init_maxwellian(prim)
        s.step(2, dt=dt)
        torch.cuda.synchronize()
        out = (s.f_canonical().cpu().numpy(), s.moments().cpu().numpy())
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), g


@pytest.mark.parametrize("nv,precision", [(24, D.PREC_FP64), (24, D.PREC_FP32), (16, D.PREC_FP64),
                                          (12, D.PREC_FP32)])
def test_every_compiled_shape_matches_oracle(nv, precision):
    """Every step-kernel shape compiled for the grid (threads per workgroup,
    waves per EU; some leave lanes idle in their last velocity round), with
    and without non-temporal stores, on an octree with FINER, COARSER, wall
    and inflow faces: f and the moments against the oracle after 3 steps"""
    import torch
    bc = (I.INFLOW, I.OUTFLOW, I.WALL, I.OUTFLOW, I.PERIODIC, I.PERIODIC)
    f = balanced(I.random_forest(14, (2, 2, 2), 2, 0.3, bc))
    case = Case(f, nv, 6.0, tau_mode=I.TAU_HS, tau=0.05, inflow=(1.0, 0.9, 0.0, 0.1, 1.0), t_wall=1.1,
                fields="sines", field_args={"seed": 14})
    o = oracle_run(case, 3)
    dm, s = gpu_solver(case, precision)
    prim = prim_for(case, dm.tables()["input"])
    tol = FP64_TOL if precision == D.PREC_FP64 else FP32_TOL
    shapes = s.shapes()
    assert len(shapes) >= 1
    for (t, w) in shapes:
        for nt in (0, 1):
            s.set_shape(t, w, 64, nt)
            s.init_maxwellian(prim)
            s.step(3, dt=o["dt"])
            torch.cuda.synchronize()
            fg = s.f_canonical().double().cpu().numpy()
            em = moment_errors(s.moments().cpu().numpy(), o["mom"])
            ef = np.abs(fg - o["f"]).max() / np.abs(o["f"]).max()
            assert np.all(em <= tol) and ef <= tol, (t, w, nt, em, ef)
