"""On-device mesh adaptation against references that do not share its code:
the adapted leaf list equals flags applied leaf by leaf in Python and closed
by the oracle's 2:1 balance (its own pointer octree); the face tables built on
the device equal the host builder's, bitwise; the remapped state equals the
definition (children copy the parent's row, a coarsened parent takes the mean
of its 8 children) on seeded data and conserves sum V f for every velocity;
stepping on the adapted mesh matches the FP64 oracle."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_00707_amd import dvm as D
from paper_1503_00707_amd import inputs as I
from tests.gpu_common import Case, balanced, moment_errors, oracle_run

pytestmark = pytest.mark.gpu


def _flags(forest_sorted, rng, p_refine=0.12, p_coarsen=0.5):
    """+1 on a random tenth of the leaves, -1 on randomly chosen complete
    sibling sets (leaves listed in Morton order)"""
    lev, ijk = forest_sorted.level.astype(int), forest_sorted.ijk.astype(int)
    n = lev.size
    fl = np.zeros(n, np.int8)
    t = 0
    while t + 8 <= n:
        grp = slice(t, t + 8)
        ci = (ijk[grp, 0] & 1) | ((ijk[grp, 1] & 1) << 1) | ((ijk[grp, 2] & 1) << 2)
        same_parent = (ijk[grp] >> 1 == ijk[t] >> 1).all() and (lev[grp] == lev[t]).all() and lev[t] >= 1
        if same_parent and np.array_equal(ci, np.arange(8)):
            if rng.random() < p_coarsen:
                fl[grp] = -1
            t += 8
        else:
            t += 1
    fl[(fl == 0) & (rng.random(n) < p_refine)] = 1
    return fl


def _apply(forest_sorted, fl):
    """the flags applied leaf by leaf, then the oracle's 2:1 closure"""
    lev, ijk = [], []
    n = fl.size
    t = 0
    while t < n:
        l, c = int(forest_sorted.level[t]), forest_sorted.ijk[t]
        if fl[t] > 0:
            for q in range(8):
                lev.append(l + 1)
                ijk.append([2 * c[0] + (q & 1), 2 * c[1] + ((q >> 1) & 1), 2 * c[2] + ((q >> 2) & 1)])
            t += 1
        elif fl[t] < 0 and t + 8 <= n and (fl[t:t + 8] < 0).all() and \
                np.array_equal((forest_sorted.ijk[t:t + 8] & 1) @ np.array([1, 2, 4]), np.arange(8)) and \
                (forest_sorted.ijk[t:t + 8] >> 1 == c >> 1).all() and (forest_sorted.level[t:t + 8] == l).all():
            lev.append(l - 1)
            ijk.append(list(c >> 1))
            t += 8
        else:
            lev.append(l)
            ijk.append(list(c))
            t += 1
    f = dataclasses.replace(forest_sorted, level=np.array(lev, np.uint8), ijk=np.array(ijk, np.int32))
    return balanced(f)


def _sorted_forest(forest):
    """the leaves in the mesh's cell (Morton) order"""
    m = O.Mesh(forest)
    inp = m.tables()["input"]
    return dataclasses.replace(forest, level=forest.level[inp], ijk=forest.ijk[inp])


def _solver(forest, nv=8, precision=D.PREC_FP64):
    dm = D.Mesh(forest)
    s = D.Solver(dm, D.make_params(nv, 4.5, precision=precision, tau_or_kn=0.1))
    return dm, s


@pytest.mark.parametrize("seed,bc", [(0, "periodic"), (1, "periodic"), (2, "open")])
def test_adapted_leaves_and_tables(seed, bc):
    import torch
    bcs = (I.PERIODIC,) * 6 if bc == "periodic" else (I.INFLOW, I.OUTFLOW, I.WALL, I.OUTFLOW, I.PERIODIC, I.PERIODIC)
    f0 = _sorted_forest(balanced(I.random_forest(seed, (2, 2, 2), 3, 0.25, bcs)))
    rng = np.random.default_rng(40 + seed)
    fl = _flags(f0, rng)
    assert (fl > 0).any() and (fl < 0).any()
    dm, s = _solver(f0)
    s.init_maxwellian(I.fields("sines", I.leaf_centres(f0), seed=seed))
    f1, m1, s1 = D.adapt(s, fl)
    want = _sorted_forest(_apply(f0, fl))
    assert np.array_equal(f1.level, want.level) and np.array_equal(f1.ijk, want.ijk)
    # device-built tables == the host builder's upload, bitwise (n records of
    # 128 bytes; the buffer's 256-byte tail padding is never written)
    torch.cuda.synchronize()
    dev = s1.tables_buf.clone()
    dm2, s2 = _solver(f1)
    torch.cuda.synchronize()
    nb = 128 * s1.n
    assert s2.n == s1.n and torch.equal(dev[:nb], s2.tables_buf[:nb])
    assert m1.n_faces == dm2.n_faces and sum(m1.n_faces) == 6 * s1.n
    # the adapted mesh keeps no host face tables
    with pytest.raises(D.DvmError):
        m1.tables()
    with pytest.raises(D.DvmError):
        D.LBM(m1)


@pytest.mark.parametrize("seed", [0, 2])
def test_adapted_solver_steps_like_a_host_built_one(seed):
    """the selection list of regular cells built on the device: with the
    step split in two launches (regular cells, then the rest, 24^3 FP32) a
    solver on the adapted mesh steps bitwise like one on the host-built mesh"""
    import torch
    bcs = (I.PERIODIC,) * 6 if seed == 0 else (I.INFLOW, I.OUTFLOW, I.WALL, I.OUTFLOW, I.PERIODIC, I.PERIODIC)
    f0 = _sorted_forest(balanced(I.random_forest(seed, (2, 2, 2), 3, 0.25, bcs)))
    fl = _flags(f0, np.random.default_rng(60 + seed))
    dm, s = _solver(f0, nv=24, precision=D.PREC_FP32)
    f1, m1, s1 = D.adapt(s, fl)
    dm2 = D.Mesh(f1)
    s2 = D.Solver(dm2, D.make_params(24, 4.5, precision=D.PREC_FP32, tau_or_kn=0.1))
    prim = I.fields("sines", I.leaf_centres(f1), seed=seed)
    for x in (s1, s2):
        x.split(1)
        x.init_maxwellian(prim)
        x.step(3, cfl=0.5)
    torch.cuda.synchronize()
    assert torch.equal(s1.f_canonical(), s2.f_canonical())
    assert torch.equal(s1.moments(), s2.moments())


@pytest.mark.parametrize("precision", [D.PREC_FP64, D.PREC_FP32])
def test_remap_is_the_definition_and_conserves(precision):
    import torch
    f0 = _sorted_forest(balanced(I.random_forest(3, (2, 2, 2), 3, 0.25)))
    rng = np.random.default_rng(7)
    fl = _flags(f0, rng)
    dm, s = _solver(f0, precision=precision)
    nv = s.nv
    x = 0.5 + rng.random((s.n, nv))
    if precision == D.PREC_FP32:
        x = x.astype(np.float32).astype(np.float64)
    s.set_f_canonical(x)
    f1, m1, s1 = D.adapt(s, fl)
    got = s1.f_canonical().double().cpu().numpy()
    # the definition, leaf by leaf: find each new leaf's old cover
    L = int(max(f0.level.max(), f1.level.max()))
    def box(level, ijk):
        sh = L - int(level)
        return np.asarray(ijk, np.int64) << sh, 1 << sh
    old = [box(l, c) for l, c in zip(f0.level, f0.ijk)]
    want = np.zeros_like(got)
    for t, (l, c) in enumerate(zip(f1.level, f1.ijk)):
        lo, sz = box(l, c)
        inside = [k for k, (olo, osz) in enumerate(old)
                  if np.all(olo >= lo) and np.all(olo + osz <= lo + sz)]
        cover = [k for k, (olo, osz) in enumerate(old) if np.all(olo <= lo) and np.all(olo + osz >= lo + sz)]
        if cover:
            want[t] = x[cover[0]]
        else:
            want[t] = sum(x[k] * (old[k][1] / sz) ** 3 for k in inside)
    tol = 1e-15 if precision == D.PREC_FP64 else 1e-7
    assert np.abs(got - want).max() <= tol * np.abs(want).max()
    V0 = (f0.h0 / 2.0 ** f0.level.astype(float)) ** 3
    V1 = (f1.h0 / 2.0 ** f1.level.astype(float)) ** 3
    assert np.abs(V1 @ got - V0 @ x).max() <= (1e-14 if precision == D.PREC_FP64 else 1e-6) * (V0 @ x).max()
    # the moments buffer describes the remapped state
    torch.cuda.synchronize()
    assert np.abs(s1.mom.cpu().numpy() - s1.moments().cpu().numpy()).max() <= 1e-14 * s1.mom.abs().max().item()


def test_no_flags_is_identity_and_adapted_mesh_steps_like_the_oracle():
    import torch
    f0 = _sorted_forest(balanced(I.random_forest(4, (2, 2, 2), 3, 0.25)))
    dm, s = _solver(f0)
    s.init_maxwellian(I.fields("sines", I.leaf_centres(f0), seed=4))
    s.step(2, cfl=0.5)
    f1, m1, s1 = D.adapt(s, np.zeros(s.n, np.int8))
    assert np.array_equal(f1.level, f0.level) and np.array_equal(f1.ijk, f0.ijk)
    torch.cuda.synchronize()
    assert np.array_equal(s1.f_canonical().cpu().numpy(), s.f_canonical().cpu().numpy())
    # a solver on an adapted mesh (tables built on the device) steps like the oracle
    fl = _flags(f0, np.random.default_rng(5))
    f2, m2, s2 = D.adapt(s, fl)
    case = Case(f2, 8, 4.5, tau=0.1, fields="sines", field_args={"seed": 9})
    o = oracle_run(case, 5)
    s2.init_maxwellian(I.fields("sines", I.leaf_centres(f2), seed=9))
    s2.step(5, dt=o["dt"])
    torch.cuda.synchronize()
    assert np.all(moment_errors(s2.moments().cpu().numpy(), o["mom"]) <= 1e-12)
    fo = o["f"]
    assert np.abs(s2.f_canonical().cpu().numpy() - fo).max() <= 1e-12 * np.abs(fo).max()


@pytest.mark.parametrize("precision", [D.PREC_FP64, D.PREC_FP32])
def test_refine_everywhere_then_coarsen_back_is_the_identity(precision):
    """refining every leaf copies its row into 8 children; coarsening every
    complete sibling set back takes their mean, of identical rows: the
    original leaf list and state (the 2:1 rule holds at every stage).  The
    mean is summed in FP64: exact for FP32 rows (bitwise), within one
    rounding per addition for FP64 rows"""
    import torch
    f0 = _sorted_forest(balanced(I.random_forest(5, (2, 2, 2), 2, 0.3)))
    dm, s = _solver(f0, precision=precision)
    s.init_maxwellian(I.fields("sines", I.leaf_centres(f0), seed=5))
    s.step(2, cfl=0.5)
    torch.cuda.synchronize()
    x0 = s.f_canonical().cpu().numpy()
    f1, m1, s1 = D.adapt(s, np.ones(s.n, np.int8))
    assert s1.n == 8 * s.n and np.array_equal(np.sort(f1.level), np.sort(np.repeat(f0.level + 1, 8)))
    f2, m2, s2 = D.adapt(s1, -np.ones(s1.n, np.int8))
    assert np.array_equal(f2.level, f0.level) and np.array_equal(f2.ijk, f0.ijk)
    torch.cuda.synchronize()
    x2 = s2.f_canonical().cpu().numpy()
    if precision == D.PREC_FP32:
        assert np.array_equal(x2, x0)
    else:
        assert np.abs(x2 - x0).max() <= 4e-16 * np.abs(x0).max()


@pytest.mark.parametrize("bc", ["periodic", "open"])
def test_muscl_on_an_adapted_mesh_steps_like_the_oracle(bc):
    """MUSCL reads two face hops through the neighbours' records: a MUSCL
    solver on a mesh adapted on the device (its face tables built there)
    steps like the oracle on the same leaves (FP64, <= 1e-12)"""
    import torch
    bcs = (I.PERIODIC,) * 6 if bc == "periodic" else (I.INFLOW, I.OUTFLOW, I.WALL, I.OUTFLOW, I.PERIODIC, I.PERIODIC)
    f0 = _sorted_forest(balanced(I.random_forest(6, (2, 2, 2), 3, 0.25, bcs)))
    dm = D.Mesh(f0)
    s = D.Solver(dm, D.make_params(8, 4.5, precision=D.PREC_FP64, scheme=I.SCHEME_MUSCL, tau_or_kn=0.1))
    s.init_maxwellian(I.fields("sines", I.leaf_centres(f0), seed=6))
    fl = _flags(f0, np.random.default_rng(16))
    f1, m1, s1 = D.adapt(s, fl)
    case = Case(f1, 8, 4.5, scheme=I.SCHEME_MUSCL, tau=0.1, fields="sines", field_args={"seed": 11})
    o = oracle_run(case, 4)
    s1.init_maxwellian(I.fields("sines", I.leaf_centres(f1), seed=11))
    s1.step(4, dt=o["dt"])
    torch.cuda.synchronize()
    assert np.all(moment_errors(s1.moments().cpu().numpy(), o["mom"]) <= 1e-12)
    fo = o["f"]
    assert np.abs(s1.f_canonical().cpu().numpy() - fo).max() <= 1e-12 * np.abs(fo).max()
