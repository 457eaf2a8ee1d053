"""Batched stepping of many independent instances (one graph launch per
step) against the same instances stepped one by one through dvm_step, and
one instance against the FP64 oracle."""
import dataclasses

import numpy as np
import pytest

from paper_1503_00707_amd import dvm as D
from paper_1503_00707_amd import inputs as I
from tests.gpu_common import Case, balanced, moment_errors, oracle_run

pytestmark = pytest.mark.gpu


def _instances(seed, count, precision, grids=(8, 12, 16)):
    ws = I.batch_workloads(seed=seed, count=count, cells_lo=150, cells_hi=1200, grids=grids)
    out = []
    for w in ws:
        f = balanced(w.forest)
        out.append((w, f))
    return out


def _solver(w, f, precision):
    m = D.Mesh(f)
    t = m.tables()
    p = D.make_params(w.nv[0], w.vhi[0], precision=precision, tau_mode=w.tau_mode, tau_or_kn=w.tau_or_kn)
    s = D.Solver(m, p)
    s.init_maxwellian(I.fields(w.fields, I.leaf_centres(f)[t["input"]], **w.field_args))
    return m, s


def _state(s):
    return s.f_canonical().double().cpu().numpy(), s.moments().cpu().numpy()


def test_batch_bitwise_equals_individual_fp64():
    import torch
    inst = _instances(11, 5, D.PREC_FP64)
    batch_side = [_solver(w, f, D.PREC_FP64) for w, f in inst]
    solo_side = [_solver(w, f, D.PREC_FP64) for w, f in inst]
    b = D.Batch([s for _, s in batch_side], cfl=0.5)
    assert sum(g["instances"] for g in b.groups()) == 5
    b.step(6)
    for (_, s1), (_, s2) in zip(batch_side, solo_side):
        s2.step(6, dt=s2.dt(0.5))
    torch.cuda.synchronize()
    for (_, s1), (_, s2) in zip(batch_side, solo_side):
        f1, m1 = _state(s1)
        f2, m2 = _state(s2)
        assert np.array_equal(f1, f2)
        assert np.array_equal(m1, m2)
        rc1, g1, bad1, n1 = s1.check()
        rc2, g2, bad2, n2 = s2.check()
        assert rc1 == 0 and n1 == 6 and not bad1
        assert np.array_equal(g1, g2)
        assert np.array_equal(s1.mom.cpu().numpy(), s2.mom.cpu().numpy())


def test_batch_graph_replays_match_eager_with_work_between():
    """every replay of the recorded step graph equals the eager steps, with
    unrelated device work and synchronisations between the replays"""
    import torch
    inst = _instances(12, 4, D.PREC_FP32)
    batch_side = [_solver(w, f, D.PREC_FP32) for w, f in inst]
    solo_side = [_solver(w, f, D.PREC_FP32) for w, f in inst]
    b = D.Batch([s for _, s in batch_side])
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(4):
        b.step(1)
        junk.add_(1.0)
        junk.zero_()
        torch.cuda.synchronize()
        for (_, s1), (_, s2) in zip(batch_side, solo_side):
            s2.step(1, dt=s2.dt(0.5))
            f1, m1 = _state(s1)
            f2, m2 = _state(s2)
            assert np.array_equal(f1, f2), rep
            assert np.array_equal(s1.mom.cpu().numpy(), s2.mom.cpu().numpy()), rep


def test_batch_branches_and_chain_agree_bitwise():
    """the velocity-grid groups recorded as parallel graph branches (default)
    and as one chain advance every instance identically, replay after replay"""
    import torch
    inst = _instances(14, 6, D.PREC_FP32)
    a_side = [_solver(w, f, D.PREC_FP32) for w, f in inst]
    b_side = [_solver(w, f, D.PREC_FP32) for w, f in inst]
    ba = D.Batch([s for _, s in a_side])
    bb = D.Batch([s for _, s in b_side])
    assert len(ba.groups()) >= 2
    assert ba.branches() == 1 and bb.branches(0) == 1 and bb.branches() == 0
    for rep in range(3):
        ba.step(2)
        bb.step(2)
        torch.cuda.synchronize()
        for (_, s1), (_, s2) in zip(a_side, b_side):
            assert np.array_equal(_state(s1)[0], _state(s2)[0]), rep
            assert np.array_equal(s1.check()[1], s2.check()[1]), rep


def test_batch_picks_up_instances_stepped_alone():
    import torch
    inst = _instances(13, 3, D.PREC_FP64)
    batch_side = [_solver(w, f, D.PREC_FP64) for w, f in inst]
    solo_side = [_solver(w, f, D.PREC_FP64) for w, f in inst]
    b = D.Batch([s for _, s in batch_side])
    b.step(2)
    batch_side[1][1].step(1, dt=batch_side[1][1].dt(0.5))  # one instance advances alone
    b.step(3)
    torch.cuda.synchronize()
    for k, ((_, s1), (_, s2)) in enumerate(zip(batch_side, solo_side)):
        s2.step(6 if k == 1 else 5, dt=s2.dt(0.5))
        f1, _ = _state(s1)
        f2, _ = _state(s2)
        assert np.array_equal(f1, f2), k


def test_batch_tune_keeps_state_and_matches():
    import torch
    inst = _instances(14, 4, D.PREC_FP32, grids=(8, 12))
    batch_side = [_solver(w, f, D.PREC_FP32) for w, f in inst]
    solo_side = [_solver(w, f, D.PREC_FP32) for w, f in inst]
    b = D.Batch([s for _, s in batch_side])
    before = [_state(s) for _, s in batch_side]
    b.tune(reps=2)
    after = [_state(s) for _, s in batch_side]
    for (f0, m0), (f1, m1) in zip(before, after):
        assert np.array_equal(f0, f1)
        assert np.abs(m1 - m0).max() <= 1e-12 * np.abs(m0).max()
    for g in b.groups():
        assert g["tuned_ms"] > 0 and g["threads"] > 0
    b.step(4)
    torch.cuda.synchronize()
    for (_, s1), (_, s2) in zip(batch_side, solo_side):
        s2.step(4, dt=s2.dt(0.5))
        _, m1 = _state(s1)
        _, m2 = _state(s2)
        assert np.all(moment_errors(m1, m2) <= 2e-6)


@pytest.mark.parametrize("precision,tol", [(D.PREC_FP64, 1e-12), (D.PREC_FP32, 2e-5)])
def test_batch_instance_matches_oracle(precision, tol):
    """every instance of a batch (grids 8^3, 12^3, 16^3) against the FP64
    oracle after 5 batched steps: moments, the global sums the batch graph
    computed (reported by dvm_check) and f"""
    import torch
    from tests.test_gpu_parity import sums_errors
    inst = _instances(15, 3, precision)
    sides = [_solver(w, f, precision) for w, f in inst]
    b = D.Batch([s for _, s in sides])
    b.step(5)
    torch.cuda.synchronize()
    for (w, f), (_, s) in zip(inst, sides):
        case = Case(f, w.nv[0], w.vhi[0], tau_mode=w.tau_mode, tau=w.tau_or_kn, fields=w.fields,
                    field_args=w.field_args)
        o = oracle_run(case, 5)
        assert s.dt(0.5) == pytest.approx(o["dt"], rel=1e-15)
        fg, mg = _state(s)
        assert np.all(moment_errors(mg, o["mom"]) <= tol)
        assert np.abs(fg - o["f"]).max() <= tol * np.abs(o["f"]).max()
        rc, sums, bad, n = s.check()
        assert rc == 0 and not bad and n == 5
        assert np.all(sums_errors(sums, o["sums"], o["mom"]) <= tol)
