"""Host-side checks of libdvm.so that need no GPU: the library loads and
exports every declared entry point; its linear-octree mesh builder agrees bit
for bit with the oracle's pointer octree; argument errors come back as status
codes."""
import dataclasses
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_00707_amd import dvm as D
from paper_1503_00707_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(dvm_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_exports_every_declared_symbol():
    L = D.lib()
    names = declared_symbols()
    assert len(names) >= 19
    for name in names:
        assert hasattr(L, name), name
    assert set(D.EXPORTED) <= set(names)


def balanced_both(forest):
    lo, io = O.balance(forest)
    ld, id_ = D.balance(forest)
    return (lo, io), (ld, id_)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("periodic", [True, False])
def test_balance_bit_exact_vs_oracle(seed, periodic):
    bc = (I.PERIODIC,) * 6 if periodic else (I.OUTFLOW,) * 6
    f = I.random_forest(seed, (2, 3, 2), 3, 0.2, bc)
    (lo, io), (ld, id_) = balanced_both(f)
    assert np.array_equal(lo, ld)
    assert np.array_equal(io, id_)


def _compare_tables(f, solid=None):
    om = O.Mesh(f, solid)
    dm = D.Mesh(f, solid)
    ot, dt = om.tables(), dm.tables()
    assert om.n_cells == dm.n_cells
    assert np.array_equal(ot["input"], dt["input"])
    assert np.array_equal(ot["key"], dt["key"])
    assert np.array_equal(ot["type"], dt["type"])
    assert np.array_equal(ot["nbr"], dt["nbr"])
    return dm


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("bc", [(I.PERIODIC,) * 6, (I.INFLOW, I.OUTFLOW, I.WALL, I.OUTFLOW, I.PERIODIC, I.PERIODIC)])
def test_tables_bit_exact_vs_oracle(seed, bc):
    f = I.random_forest(seed, (2, 2, 3), 3, 0.2, bc)
    lev, ijk = D.balance(f)
    _compare_tables(dataclasses.replace(f, level=lev, ijk=ijk))


def test_tables_bit_exact_sphere_with_solid():
    f = I.sphere_refinement(base=(8, 8, 8), levels=2, radius=0.2)
    lev, ijk = D.balance(f)
    fb = dataclasses.replace(f, level=lev, ijk=ijk)
    sol = I.solid_flags(fb, (0.5, 0.5, 0.5), 0.2, 2)
    dm = _compare_tables(fb, sol)
    assert dm.n_faces[D.ERR_ARG + 6] >= 0  # smoke
    assert dm.n_cells == fb.n - int(sol.sum())


def test_tables_bit_exact_random_roots_16():
    f = I.random_root_refinement((16, 16, 16), 0.4, 3, h0=1 / 16)
    _compare_tables(f)


def test_argument_errors():
    f = I.random_forest(0, (2, 2, 2), 3, 0.3)
    with pytest.raises(D.DvmError) as e:
        D.Mesh(f)
    assert e.value.code == D.ERR_UNBALANCED
    g = I.uniform_forest((2, 2, 2), 1)
    with pytest.raises(D.DvmError) as e:
        D.Mesh(dataclasses.replace(g, level=g.level[1:], ijk=g.ijk[1:]))
    assert e.value.code == D.ERR_NOT_PARTITION
    dup = dataclasses.replace(g, level=np.concatenate([g.level, g.level[:1]]), ijk=np.concatenate([g.ijk, g.ijk[:1]]))
    with pytest.raises(D.DvmError) as e:
        D.Mesh(dup)
    assert e.value.code == D.ERR_NOT_PARTITION
    with pytest.raises(D.DvmError) as e:
        D.Mesh(dataclasses.replace(g, bc=(I.PERIODIC, I.OUTFLOW) + (I.PERIODIC,) * 4))
    assert e.value.code == D.ERR_ARG
    with pytest.raises(D.DvmError) as e:  # no leaves at all
        D.Mesh(dataclasses.replace(g, level=g.level[:0], ijk=g.ijk[:0]))
    assert e.value.code == D.ERR_ARG


def test_solver_argument_errors_host_only():
    m = D.Mesh(I.uniform_forest((1, 1, 1), 2))
    import ctypes as C
    h = C.c_void_p()
    for p, code in [(D.make_params(7, 4.5), D.ERR_UNSUPPORTED), (D.make_params(10, 4.5), D.ERR_UNSUPPORTED),
                    (D.make_params(8, -1.0), D.ERR_ARG), (D.make_params(8, 4.5, tau_or_kn=0.0), D.ERR_ARG)]:
        assert D.lib().dvm_create_solver(m.h, C.byref(p), C.byref(h)) == code
    p = D.make_params(8, 4.5)
    assert D.lib().dvm_create_solver(m.h, C.byref(p), C.byref(h)) == D.OK
    sz = D.Sizes()
    assert D.lib().dvm_buffer_sizes(h, C.byref(sz)) == D.OK
    assert sz.n_cells == 64 and sz.nv_total == 512 and sz.f_bytes == 64 * 512 * 4
    # step before bind/upload is refused before any device call
    assert D.lib().dvm_step(h, 1, 0.0, 0.5, None) == D.ERR_WORKSPACE
    dt = C.c_double()
    assert D.lib().dvm_dt(h, C.c_double(0.5), C.byref(dt)) == D.OK
    assert dt.value == 0.5 * 0.25 / (3 * 3.9375)
    D.lib().dvm_destroy_solver(h)


def test_muscl_solver_workspace_host_only():
    """MUSCL reconstructs its face values inside the step: the buffers are
    those of the first-order scheme (no face-value planes)"""
    import ctypes as C
    m = D.Mesh(I.uniform_forest((1, 1, 1), 2))
    sizes = {}
    for scheme in (D.SCHEME_UPWIND1, D.SCHEME_MUSCL):
        h = C.c_void_p()
        p = D.make_params(8, 4.5, scheme=scheme)
        assert D.lib().dvm_create_solver(m.h, C.byref(p), C.byref(h)) == D.OK
        sz = D.Sizes()
        assert D.lib().dvm_buffer_sizes(h, C.byref(sz)) == D.OK
        sizes[scheme] = (sz.f_bytes, sz.ws_bytes)
        D.lib().dvm_destroy_solver(h)
    assert sizes[D.SCHEME_MUSCL] == sizes[D.SCHEME_UPWIND1]


def test_batch_create_errors_host_only():
    """dvm_batch_create groups host solvers and rejects what the batched
    kernel does not do; no device call happens before dvm_batch_bind"""
    import ctypes as C
    m = D.Mesh(I.uniform_forest((1, 1, 1), 2))
    hs = []
    for nv, prec, scheme in [(8, D.PREC_FP32, D.SCHEME_UPWIND1), (12, D.PREC_FP32, D.SCHEME_UPWIND1),
                             (8, D.PREC_FP64, D.SCHEME_UPWIND1), (8, D.PREC_FP32, D.SCHEME_MUSCL)]:
        h = C.c_void_p()
        p = D.make_params(nv, 4.5, precision=prec, scheme=scheme)
        assert D.lib().dvm_create_solver(m.h, C.byref(p), C.byref(h)) == D.OK
        hs.append(h)
    arr = lambda *xs: (C.c_void_p * len(xs))(*[x.value for x in xs])
    b = C.c_void_p()
    assert D.lib().dvm_batch_create(arr(hs[0]), 0, 0.5, C.byref(b)) == D.ERR_ARG
    assert D.lib().dvm_batch_create(arr(hs[0], hs[0]), 2, 0.5, C.byref(b)) == D.ERR_ARG
    assert D.lib().dvm_batch_create(arr(hs[0], hs[2]), 2, 0.5, C.byref(b)) == D.ERR_UNSUPPORTED
    assert D.lib().dvm_batch_create(arr(hs[0], hs[3]), 2, 0.5, C.byref(b)) == D.ERR_UNSUPPORTED
    assert D.lib().dvm_batch_create(arr(hs[0], hs[1]), 2, -1.0, C.byref(b)) == D.ERR_ARG
    assert D.lib().dvm_batch_create(arr(hs[0], hs[1]), 2, 0.5, C.byref(b)) == D.OK
    nb = C.c_size_t(0)
    assert D.lib().dvm_batch_workspace_bytes(b, C.byref(nb)) == D.OK and nb.value > 0
    ng = C.c_int32(0)
    assert D.lib().dvm_batch_info(b, -1, None, C.byref(ng), None, None, None, None, None, None) == D.OK
    assert ng.value == 2  # two velocity grids
    nh, ni, cells = C.c_int32(), C.c_int32(), C.c_int64()
    assert D.lib().dvm_batch_info(b, 0, C.byref(nh), C.byref(ni), C.byref(cells), None, None, None, None,
                                  None) == D.OK
    assert (nh.value, ni.value, cells.value) == (6, 1, 64)  # larger grid first
    assert D.lib().dvm_batch_step(b, 1, None) == D.ERR_WORKSPACE  # not bound
    D.lib().dvm_destroy_batch(b)
    for h in hs:
        D.lib().dvm_destroy_solver(h)


def test_split_setting_host_only():
    """the regular/irregular split is off by default, can be queried and turned
    on, and rejects a shape that was not compiled; no device call"""
    import ctypes as C
    m = D.Mesh(I.uniform_forest((1, 1, 1), 2))
    h = C.c_void_p()
    p = D.make_params(24, 6.0)
    assert D.lib().dvm_create_solver(m.h, C.byref(p), C.byref(h)) == D.OK
    prev = C.c_int32(-7)
    assert D.lib().dvm_tune_split(h, -1, 0, 0, C.byref(prev)) == D.OK and prev.value == 0
    assert D.lib().dvm_tune_split(h, 1, 0, 0, C.byref(prev)) == D.OK and prev.value == 0
    assert D.lib().dvm_tune_split(h, -1, 0, 0, C.byref(prev)) == D.OK and prev.value == 1
    assert D.lib().dvm_tune_split(h, 1, 100, 31, None) == D.ERR_UNSUPPORTED
    assert D.lib().dvm_tune_split(h, 1, 576, 71, None) == D.OK
    D.lib().dvm_destroy_solver(h)


def test_tuner_cache_file_round_trip(tmp_path):
    """the tuner cache (dvm_tune, dvm_batch_tune) keeps one line per key and
    returns what was stored; a replaced key keeps one line; other keys and
    unreadable lines survive; a missing file or key is not found"""
    path = str(tmp_path / "tune.txt")
    assert D.tune_cache_get(path, "step", "gfx950", 12, 0, 0) is None
    D.tune_cache_put(path, "step", "gfx950", 12, 0, 0, (192, 31, 512, 1), 29.5)
    D.tune_cache_put(path, "batch", "gfx950", 6, 0, 0, (128, 60, 64, 1), 7.25)
    D.tune_cache_put(path, "step", "gfx950", 12, 1, 0, (576, 30, 64, 1), 85.0)
    with open(path, "a") as fh:
        fh.write("not a cache line\n")
    assert D.tune_cache_get(path, "step", "gfx950", 12, 0, 0) == ((192, 31, 512, 1), 29.5)
    assert D.tune_cache_get(path, "batch", "gfx950", 6, 0, 0) == ((128, 60, 64, 1), 7.25)
    assert D.tune_cache_get(path, "step", "gfx950", 12, 1, 0) == ((576, 30, 64, 1), 85.0)
    assert D.tune_cache_get(path, "step", "gfx942", 12, 0, 0) is None      # another architecture
    assert D.tune_cache_get(path, "step", "gfx950", 12, 0, 1) is None      # another scheme
    assert D.tune_cache_get(path, "batch", "gfx950", 12, 0, 0) is None     # another kind
    D.tune_cache_put(path, "step", "gfx950", 12, 0, 0, (256, 0, 64, 0), 31.0)
    assert D.tune_cache_get(path, "step", "gfx950", 12, 0, 0) == ((256, 0, 64, 0), 31.0)
    lines = open(path).read().splitlines()
    assert sum(line.startswith("step gfx950 nh=12 fp64=0 scheme=0 |") for line in lines) == 1
    assert "not a cache line" in lines and len(lines) == 4
    with pytest.raises(D.DvmError):
        D.tune_cache_put(path, "other", "gfx950", 12, 0, 0, (256, 0, 64, 0), 1.0)


@pytest.mark.parametrize("nv,vmax,p", [(4, 3.0, 31), (8, 4.5, 127), (8, 4.5, 1021), (12, 6.0, 61)])
def test_korobov_tables_bit_exact_vs_oracle(nv, vmax, p):
    """the library's Korobov generator and trial tables (built on the host by
    its own code) equal the oracle's, bit for bit"""
    a = D.korobov_generator(p)
    assert a == O.korobov_generator(p)
    j, l, m = D.korobov_tables(nv, vmax, p, a)
    jo, lo, mo, _ = O.korobov_tables((nv,) * 3, (-vmax,) * 3, (vmax,) * 3, p, a)
    assert np.array_equal(j, jo) and np.array_equal(l, lo) and np.array_equal(m, mo)


def test_korobov_solver_arguments_host_only():
    f = I.uniform_forest((1, 1, 1), 1)
    m = D.Mesh(f)
    for kw, code in ((dict(nv=8, korobov_p=100), D.ERR_ARG),       # not prime
                     (dict(nv=16, korobov_p=127), D.ERR_UNSUPPORTED),  # no kernel for 16^3
                     (dict(nv=8, korobov_p=127, hybrid=True), D.ERR_UNSUPPORTED)):
        nv = kw.pop("nv")
        p = D.make_params(nv, 4.5, collision=D.COLL_KOROBOV, tau_or_kn=0.5, **kw)
        h = __import__("ctypes").c_void_p()
        assert D.lib().dvm_create_solver(m.h, __import__("ctypes").byref(p), __import__("ctypes").byref(h)) == code


def test_one_hip_runtime_in_the_process():
    """the library shares torch's HIP runtime: after loading it, exactly one
    HIP runtime is mapped, whichever of the two was asked for first (streams
    and events handed over by torch belong to the runtime that launches)"""
    import subprocess
    import sys
    code = ("from paper_1503_00707_amd import dvm as D; D.lib(); import torch; "
            "print(sorted(set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l)))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__)))).stdout
    libs = eval(out.strip().splitlines()[-1])
    assert len(libs) == 1, libs
