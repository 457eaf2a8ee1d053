"""ctypes binding of libdvm.so (include/dvm.h): argument marshalling only.

Every step of the DVM path runs in the HIP library; PyTorch supplies device
memory (torch.empty on the GPU) and the stream.  The binding raises if the
built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdvm.so")

OK, ERR_ARG, ERR_UNBALANCED, ERR_NOT_PARTITION, ERR_WORKSPACE, ERR_NONPHYSICAL, ERR_DEVICE, ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
PREC_FP64, PREC_FP32 = 0, 1
SCHEME_UPWIND1, SCHEME_MUSCL = 0, 1
COLL_EXP, COLL_EULER, COLL_OFF, COLL_KOROBOV = 0, 1, 2, 3
TAU_CONST, TAU_HS = 0, 1
FLUX_GRID, FLUX_CLOSED = 0, 1

EXPORTED = [
    "dvm_last_error", "dvm_balance", "dvm_create_mesh", "dvm_mesh_info", "dvm_mesh_export", "dvm_destroy_mesh",
    "dvm_create_solver", "dvm_buffer_sizes", "dvm_bind", "dvm_upload", "dvm_init_maxwellian", "dvm_step",
    "dvm_dt", "dvm_global_sums", "dvm_current_f", "dvm_moments", "dvm_check", "dvm_f_to_canonical", "dvm_f_from_canonical",
    "dvm_destroy_solver", "dvm_tune_shapes", "dvm_tune_set", "dvm_tune_get", "dvm_tune_split",
    "dvm_batch_create", "dvm_batch_workspace_bytes", "dvm_batch_bind", "dvm_batch_step", "dvm_batch_tune",
    "dvm_batch_info", "dvm_destroy_batch",
    "dvm_features", "dvm_labels", "dvm_mlp_create", "dvm_mlp_workspace_bytes", "dvm_mlp_bind",
    "dvm_mlp_set_normalization", "dvm_mlp_forward", "dvm_mlp_gradient", "dvm_mlp_adam", "dvm_mlp_train_step",
    "dvm_mlp_buffers", "dvm_destroy_mlp", "dvm_sensor", "dvm_hybrid_step",
    "dvm_tune", "dvm_save", "dvm_load", "dvm_tune_cache_get", "dvm_tune_cache_put",
    "dvm_mlp_gradient_noalloc", "dvm_korobov_generator", "dvm_korobov_tables",
    "dvm_batch_branches", "dvm_adapt_workspace_bytes", "dvm_adapt_leaves", "dvm_adapt_mesh", "dvm_adapt_tables", "dvm_adapt_remap",
    "dvm_lbm_create", "dvm_lbm_buffer_sizes", "dvm_lbm_bind", "dvm_lbm_upload", "dvm_lbm_init", "dvm_lbm_dt",
    "dvm_lbm_step", "dvm_lbm_moments", "dvm_lbm_check", "dvm_lbm_get_f", "dvm_lbm_set_f", "dvm_lbm_current_f",
    "dvm_destroy_lbm",
]
MLP_WEIGHTS, MLP_PARAMS = 4929, 4949


class DvmError(RuntimeError):
    def __init__(self, code: int, what: str, text: str):
        super().__init__(f"{what} failed with {code}: {text}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("base", C.c_int32 * 3), ("h0", C.c_double), ("bc", C.c_int32 * 6), ("n_leaves", C.c_int64),
                ("level", C.c_void_p), ("ijk", C.c_void_p), ("solid", C.c_void_p)]


class MeshInfo(C.Structure):
    _fields_ = [("n_leaves", C.c_int64), ("n_cells", C.c_int64), ("max_level", C.c_int32), ("h_min", C.c_double),
                ("n_faces", C.c_int64 * 6)]


class Params(C.Structure):
    _fields_ = [("nv", C.c_int32), ("vmax", C.c_double * 3), ("precision", C.c_int32), ("scheme", C.c_int32),
                ("collision", C.c_int32), ("tau_mode", C.c_int32), ("tau_or_kn", C.c_double),
                ("inflow", C.c_double * 5), ("t_wall", C.c_double), ("check_every", C.c_int32),
                ("hybrid", C.c_int32), ("korobov_p", C.c_int32), ("korobov_a", C.c_int32),
                ("fluid_flux", C.c_int32)]


class LbmParams(C.Structure):
    _fields_ = [("q", C.c_int32), ("precision", C.c_int32), ("collision", C.c_int32), ("tau", C.c_double)]


class Sizes(C.Structure):
    _fields_ = [("f_bytes", C.c_size_t), ("moments_bytes", C.c_size_t), ("tables_bytes", C.c_size_t),
                ("ws_bytes", C.c_size_t), ("n_cells", C.c_int64), ("nv_total", C.c_int64)]


class Diag(C.Structure):
    _fields_ = [("sums", C.c_double * 5), ("nonphysical", C.c_int32), ("steps", C.c_int64)]


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1503_00707_amd.build`")
        # torch first: the library then resolves its HIP runtime to the one
        # torch loaded (same soname), so the streams and device buffers torch
        # hands over belong to the runtime that launches the kernels; loaded
        # first, it would bring a second runtime into the process
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.dvm_last_error.restype = C.c_char_p
        L.dvm_balance.argtypes = [C.POINTER(MeshDesc), C.c_int64, C.POINTER(C.c_int64), P, P]
        L.dvm_create_mesh.argtypes = [C.POINTER(MeshDesc), C.POINTER(P)]
        L.dvm_mesh_info.argtypes = [P, C.POINTER(MeshInfo)]
        L.dvm_mesh_export.argtypes = [P, P, P, P, P]
        L.dvm_destroy_mesh.argtypes = [P]
        L.dvm_destroy_mesh.restype = None
        L.dvm_create_solver.argtypes = [P, C.POINTER(Params), C.POINTER(P)]
        L.dvm_buffer_sizes.argtypes = [P, C.POINTER(Sizes)]
        L.dvm_bind.argtypes = [P, P, P, P, P, P]
        L.dvm_upload.argtypes = [P, P]
        L.dvm_init_maxwellian.argtypes = [P, P, P]
        L.dvm_step.argtypes = [P, C.c_int32, C.c_double, C.c_double, P]
        L.dvm_dt.argtypes = [P, C.c_double, C.POINTER(C.c_double)]
        L.dvm_global_sums.argtypes = [P, P]
        L.dvm_current_f.argtypes = [P, C.POINTER(P)]
        L.dvm_moments.argtypes = [P, P, P]
        L.dvm_check.argtypes = [P, P, C.POINTER(Diag)]
        L.dvm_f_to_canonical.argtypes = [P, P, P, P]
        L.dvm_f_from_canonical.argtypes = [P, P, P, P]
        L.dvm_tune_shapes.argtypes = [P, P, P, C.c_int32, C.POINTER(C.c_int32)]
        L.dvm_tune_set.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.dvm_tune_get.argtypes = [P, P, P, P, P]
        L.dvm_tune_split.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
        L.dvm_destroy_solver.argtypes = [P]
        L.dvm_destroy_solver.restype = None
        L.dvm_batch_create.argtypes = [P, C.c_int32, C.c_double, C.POINTER(P)]
        L.dvm_batch_workspace_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
        L.dvm_batch_bind.argtypes = [P, P]
        L.dvm_batch_step.argtypes = [P, C.c_int32, P]
        L.dvm_batch_tune.argtypes = [P, C.c_int32, C.c_char_p, P]
        L.dvm_tune.argtypes = [P, C.c_char_p, C.c_int32, C.POINTER(C.c_int32), P]
        L.dvm_save.argtypes = [P, P, C.c_char_p, P]
        L.dvm_load.argtypes = [P, P, C.c_char_p, P]
        L.dvm_adapt_workspace_bytes.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
        L.dvm_adapt_leaves.argtypes = [P, P, C.c_int64, P, P, C.POINTER(C.c_int64), P, C.c_size_t, P]
        L.dvm_adapt_mesh.argtypes = [P, P, P, C.c_int64, C.POINTER(P), P]
        L.dvm_adapt_tables.argtypes = [P, P, P, P, C.c_size_t, P]
        L.dvm_adapt_remap.argtypes = [P, P, P, C.c_size_t, P]
        L.dvm_batch_branches.argtypes = [P, C.c_int32, C.POINTER(C.c_int32)]
        L.dvm_lbm_create.argtypes = [P, C.POINTER(LbmParams), C.POINTER(P)]
        L.dvm_lbm_buffer_sizes.argtypes = [P, C.POINTER(Sizes)]
        L.dvm_lbm_bind.argtypes = [P, P, P, P, P, P]
        L.dvm_lbm_upload.argtypes = [P, P]
        L.dvm_lbm_init.argtypes = [P, P, P]
        L.dvm_lbm_dt.argtypes = [P, C.c_double, C.POINTER(C.c_double)]
        L.dvm_lbm_step.argtypes = [P, C.c_int32, C.c_double, C.c_double, P]
        L.dvm_lbm_moments.argtypes = [P, P, P]
        L.dvm_lbm_check.argtypes = [P, P, C.POINTER(Diag)]
        L.dvm_lbm_get_f.argtypes = [P, P, P]
        L.dvm_lbm_set_f.argtypes = [P, P, P]
        L.dvm_lbm_current_f.argtypes = [P, C.POINTER(P)]
        L.dvm_destroy_lbm.argtypes = [P]
        L.dvm_destroy_lbm.restype = None
        L.dvm_korobov_generator.argtypes = [C.c_int64, C.POINTER(C.c_int64)]
        L.dvm_korobov_tables.argtypes = [C.c_int32, C.c_double, C.c_int64, C.c_int64, P, P, P]
        L.dvm_mlp_gradient_noalloc.argtypes = [P, P, P, C.c_int64, C.c_float, P, P, P]
        L.dvm_tune_cache_get.argtypes = [C.c_char_p, C.c_char_p, C.c_char_p, C.c_int32, C.c_int32, C.c_int32, P,
                                         C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.dvm_tune_cache_put.argtypes = [C.c_char_p, C.c_char_p, C.c_char_p, C.c_int32, C.c_int32, C.c_int32, P,
                                         C.c_double]
        L.dvm_batch_info.argtypes = [P, C.c_int32, P, P, P, P, P, P, P, P]
        L.dvm_destroy_batch.argtypes = [P]
        L.dvm_destroy_batch.restype = None
        L.dvm_features.argtypes = [P, P, P]
        L.dvm_labels.argtypes = [P, P, P]
        L.dvm_mlp_create.argtypes = [C.c_int64, C.POINTER(P)]
        L.dvm_mlp_workspace_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
        L.dvm_mlp_bind.argtypes = [P, P, P]
        L.dvm_mlp_set_normalization.argtypes = [P, P, C.c_int64, P]
        L.dvm_mlp_forward.argtypes = [P, P, C.c_int64, C.c_int32, P, P]
        L.dvm_mlp_gradient.argtypes = [P, P, P, C.c_int64, C.c_float, P]
        L.dvm_mlp_adam.argtypes = [P, C.c_float, P]
        L.dvm_mlp_train_step.argtypes = [P, P, P, C.c_int64, C.c_float, C.c_float, P]
        L.dvm_mlp_buffers.argtypes = [P, C.POINTER(P), C.POINTER(P)]
        L.dvm_destroy_mlp.argtypes = [P]
        L.dvm_destroy_mlp.restype = None
        L.dvm_sensor.argtypes = [P, P, C.c_double, P, P, P]
        L.dvm_hybrid_step.argtypes = [P, P, C.c_int32, C.c_double, C.c_double, P]
        _LIB = L
    return _LIB


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise DvmError(rc, what, lib().dvm_last_error().decode())


def _desc(forest, solid=None):
    lev = np.ascontiguousarray(forest.level, np.uint8)
    ijk = np.ascontiguousarray(forest.ijk, np.int32).reshape(-1)
    sol = None if solid is None else np.ascontiguousarray(solid, np.uint8)
    d = MeshDesc()
    for a in range(3):
        d.base[a] = int(forest.base[a])
    d.h0 = float(forest.h0)
    for f in range(6):
        d.bc[f] = int(forest.bc[f])
    d.n_leaves = int(lev.shape[0])
    d.level = lev.ctypes.data
    d.ijk = ijk.ctypes.data
    d.solid = None if sol is None else sol.ctypes.data
    return d, (lev, ijk, sol)


def balance(forest):
    """2:1 balance (faces, edges, corners); returns (level, ijk) in Morton order."""
    d, keep = _desc(forest)
    n = C.c_int64(0)
    rc = lib().dvm_balance(C.byref(d), 0, C.byref(n), None, None)
    if rc not in (OK, ERR_WORKSPACE):
        _check(rc, "dvm_balance")
    lev = np.zeros(n.value, np.uint8)
    ijk = np.zeros((n.value, 3), np.int32)
    _check(lib().dvm_balance(C.byref(d), n.value, C.byref(n), lev.ctypes.data, ijk.ctypes.data), "dvm_balance")
    return lev, ijk


class Mesh:
    def __init__(self, forest, solid: Optional[np.ndarray] = None):
        d, keep = _desc(forest, solid)
        h = C.c_void_p()
        _check(lib().dvm_create_mesh(C.byref(d), C.byref(h)), "dvm_create_mesh")
        self.h = h
        self.forest = forest
        self._info()

    @classmethod
    def wrap(cls, h, forest):
        """a Mesh object owning the handle `h` (e.g. from dvm_adapt_mesh)"""
        self = cls.__new__(cls)
        self.h, self.forest = h, forest
        self._info()
        return self

    def _info(self):
        info = MeshInfo()
        _check(lib().dvm_mesh_info(self.h, C.byref(info)), "dvm_mesh_info")
        self.n_leaves, self.n_cells = int(info.n_leaves), int(info.n_cells)
        self.h_min, self.max_level = float(info.h_min), int(info.max_level)
        self.n_faces = list(info.n_faces)

    def tables(self):
        n = self.n_cells
        inp = np.zeros(n, np.int64)
        key = np.zeros(n, np.uint64)
        ty = np.zeros((n, 6), np.uint8)
        nb = np.zeros((n, 6, 4), np.int32)
        _check(lib().dvm_mesh_export(self.h, inp.ctypes.data, key.ctypes.data, ty.ctypes.data, nb.ctypes.data),
               "dvm_mesh_export")
        return dict(input=inp, key=key, type=ty, nbr=nb)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().dvm_destroy_mesh(self.h)
                self.h = None
        except Exception:  # interpreter shutdown
            pass


def make_params(nv, vmax, precision=PREC_FP32, scheme=SCHEME_UPWIND1, collision=COLL_EXP, tau_mode=TAU_CONST,
                tau_or_kn=0.1, inflow=(1.0, 0.0, 0.0, 0.0, 1.0), t_wall=1.0, check_every=0,
                hybrid=False, korobov_p=0, korobov_a=0, fluid_flux=0) -> Params:
    p = Params()
    p.nv = int(nv)
    vm = (vmax,) * 3 if np.isscalar(vmax) else tuple(vmax)
    for a in range(3):
        p.vmax[a] = float(vm[a])
    p.precision, p.scheme, p.collision, p.tau_mode = int(precision), int(scheme), int(collision), int(tau_mode)
    p.tau_or_kn = float(tau_or_kn)
    for a in range(5):
        p.inflow[a] = float(inflow[a])
    p.t_wall = float(t_wall)
    p.check_every = int(check_every)
    p.hybrid = int(bool(hybrid))
    p.korobov_p, p.korobov_a = int(korobov_p), int(korobov_a)
    p.fluid_flux = int(fluid_flux)
    return p


def korobov_generator(p):
    """Korobov's optimal generator of a p-point lattice in 5 dimensions (dvm_korobov_generator)"""
    a = C.c_int64(0)
    _check(lib().dvm_korobov_generator(int(p), C.byref(a)), "dvm_korobov_generator")
    return a.value


def korobov_tables(nv, vmax, p, a):
    """(j, l, m) [N^3, p] of the Korobov collision tables, canonical velocity order"""
    n = int(nv) ** 3 * int(p)
    j, l, m = (np.zeros(n, np.int32) for _ in range(3))
    _check(lib().dvm_korobov_tables(int(nv), float(vmax), int(p), int(a), j.ctypes.data, l.ctypes.data,
                                    m.ctypes.data), "dvm_korobov_tables")
    sh = (int(nv) ** 3, int(p))
    return j.reshape(sh), l.reshape(sh), m.reshape(sh)


def tune_cache_get(path, kind, arch, nh, fp64, scheme):
    """(threads, wpe, xcd_group, nt_store), ms) stored for the key, or None"""
    shape = np.zeros(4, np.int32)
    ms = C.c_double(0)
    found = C.c_int32(0)
    _check(lib().dvm_tune_cache_get(os.fsencode(path), kind.encode(), arch.encode(), int(nh), int(fp64), int(scheme),
                                    shape.ctypes.data, C.byref(ms), C.byref(found)), "dvm_tune_cache_get")
    return (tuple(int(x) for x in shape), ms.value) if found.value else None


def tune_cache_put(path, kind, arch, nh, fp64, scheme, shape, ms):
    sh = np.ascontiguousarray(shape, np.int32)
    _check(lib().dvm_tune_cache_put(os.fsencode(path), kind.encode(), arch.encode(), int(nh), int(fp64), int(scheme),
                                    sh.ctypes.data, float(ms)), "dvm_tune_cache_put")


class Solver:
    """Owns the torch device buffers of one solver and drives the C interface."""

    def __init__(self, mesh: Mesh, params: Params, device="cuda"):
        import torch
        self.torch = torch
        self.mesh = mesh
        self.params = params
        h = C.c_void_p()
        _check(lib().dvm_create_solver(mesh.h, C.byref(params), C.byref(h)), "dvm_create_solver")
        self.h = h
        sz = Sizes()
        _check(lib().dvm_buffer_sizes(h, C.byref(sz)), "dvm_buffer_sizes")
        self.sizes = sz
        self.n, self.nv = int(sz.n_cells), int(sz.nv_total)
        self.fdtype = torch.float64 if params.precision == PREC_FP64 else torch.float32
        dev = torch.device(device)

        def buf(nbytes):  # 256-byte aligned: the caching allocator aligns to 512
            return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)

        self.f_a, self.f_b = buf(sz.f_bytes), buf(sz.f_bytes)
        self.mom = torch.empty((5, self.n), dtype=torch.float64, device=dev)
        self.tables_buf = buf(sz.tables_bytes)
        self.ws = buf(sz.ws_bytes)
        _check(lib().dvm_bind(h, self.f_a.data_ptr(), self.f_b.data_ptr(), self.mom.data_ptr(),
                              self.tables_buf.data_ptr(), self.ws.data_ptr()), "dvm_bind")
        _check(lib().dvm_upload(h, self.stream()), "dvm_upload")

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def init_maxwellian(self, prim):
        t = self.torch.as_tensor(np.ascontiguousarray(prim, np.float64)).to("cuda")
        self._prim = t
        _check(lib().dvm_init_maxwellian(self.h, t.data_ptr(), self.stream()), "dvm_init_maxwellian")

    def step(self, n=1, dt=0.0, cfl=0.5):
        _check(lib().dvm_step(self.h, int(n), float(dt), float(cfl), self.stream()), "dvm_step")

    def global_sums(self):
        _check(lib().dvm_global_sums(self.h, self.stream()), "dvm_global_sums")

    def dt(self, cfl):
        out = C.c_double()
        _check(lib().dvm_dt(self.h, float(cfl), C.byref(out)), "dvm_dt")
        return out.value

    def current(self):
        p = C.c_void_p()
        _check(lib().dvm_current_f(self.h, C.byref(p)), "dvm_current_f")
        return self.f_a if p.value == self.f_a.data_ptr() else self.f_b

    def f_canonical(self):
        """current state as a [n, N^3] torch tensor in canonical velocity order"""
        out = self.torch.empty((self.n, self.nv), dtype=self.fdtype, device="cuda")
        _check(lib().dvm_f_to_canonical(self.h, self.current().data_ptr(), out.data_ptr(), self.stream()),
               "dvm_f_to_canonical")
        return out

    def set_f_canonical(self, f):
        t = self.torch.as_tensor(np.ascontiguousarray(f)).to(device="cuda", dtype=self.fdtype)
        _check(lib().dvm_f_from_canonical(self.h, t.data_ptr(), self.current().data_ptr(), self.stream()),
               "dvm_f_from_canonical")
        self.torch.cuda.synchronize()

    def moments(self):
        out = self.torch.empty((5, self.n), dtype=self.torch.float64, device="cuda")
        _check(lib().dvm_moments(self.h, out.data_ptr(), self.stream()), "dvm_moments")
        return out

    def tune(self, cache_path=None, reps=2):
        """time the compiled kernel shapes on this solver (dvm_tune); returns
        True if the choice came from the tuner cache file"""
        fc = C.c_int32(0)
        cp = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().dvm_tune(self.h, cp, int(reps), C.byref(fc), self.stream()), "dvm_tune")
        return bool(fc.value)

    def save(self, path, net=None):
        """checkpoint: leaf list, f, moments, step count (and the network)"""
        _check(lib().dvm_save(self.h, None if net is None else net.h, os.fsencode(path), self.stream()), "dvm_save")

    def load(self, path, net=None):
        _check(lib().dvm_load(self.h, None if net is None else net.h, os.fsencode(path), self.stream()), "dvm_load")

    def check(self):
        d = Diag()
        rc = lib().dvm_check(self.h, self.stream(), C.byref(d))
        if rc not in (OK, ERR_NONPHYSICAL):
            _check(rc, "dvm_check")
        return rc, np.array(d.sums[:]), bool(d.nonphysical), int(d.steps)

    def shapes(self):
        n = C.c_int32(0)
        t = np.zeros(64, np.int32)
        w = np.zeros(64, np.int32)
        _check(lib().dvm_tune_shapes(self.h, t.ctypes.data, w.ctypes.data, 64, C.byref(n)), "dvm_tune_shapes")
        return [(int(t[k]), int(w[k])) for k in range(min(n.value, 64))]

    def set_shape(self, threads, wpe, xcd_group=1, nt_store=0):
        _check(lib().dvm_tune_set(self.h, int(threads), int(wpe), int(xcd_group), int(nt_store)), "dvm_tune_set")

    def split(self, enable=-1, threads_irr=0, wpe_irr=0):
        """cells without FINER or WALL faces in a reduced kernel (1) or every
        cell in one launch (0); <0 only queries; returns the previous setting"""
        prev = C.c_int32(0)
        _check(lib().dvm_tune_split(self.h, int(enable), int(threads_irr), int(wpe_irr), C.byref(prev)),
               "dvm_tune_split")
        return prev.value

    def features(self):
        """[n, 10] float32 sensor features of the current moments"""
        out = self.torch.empty((self.n, 10), dtype=self.torch.float32, device="cuda")
        _check(lib().dvm_features(self.h, out.data_ptr(), self.stream()), "dvm_features")
        return out

    def labels(self):
        """[n] float32 |f - Mt| / |Mt| of the current state"""
        out = self.torch.empty(self.n, dtype=self.torch.float32, device="cuda")
        _check(lib().dvm_labels(self.h, out.data_ptr(), self.stream()), "dvm_labels")
        return out

    def sensor(self, net=None, kappa=0.0):
        """(mask uint8 [n], score float32 [n]): network (net) or Kn_GLL > kappa"""
        mask = self.torch.empty(self.n, dtype=self.torch.uint8, device="cuda")
        score = self.torch.empty(self.n, dtype=self.torch.float32, device="cuda")
        _check(lib().dvm_sensor(self.h, None if net is None else net.h, float(kappa), mask.data_ptr(),
                                score.data_ptr(), self.stream()), "dvm_sensor")
        return mask, score

    def hybrid_step(self, mask, n=1, dt=0.0, cfl=0.5):
        m = self.torch.as_tensor(mask).to(device="cuda", dtype=self.torch.uint8).contiguous()
        self._mask = m
        _check(lib().dvm_hybrid_step(self.h, m.data_ptr(), int(n), float(dt), float(cfl), self.stream()),
               "dvm_hybrid_step")

    def get_shape(self):
        v = np.zeros(4, np.int32)
        _check(lib().dvm_tune_get(self.h, v[0:].ctypes.data, v[1:].ctypes.data, v[2:].ctypes.data,
                                  v[3:].ctypes.data), "dvm_tune_get")
        return tuple(int(x) for x in v)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().dvm_destroy_solver(self.h)
                self.h = None
        except Exception:  # interpreter shutdown
            pass


def adapt(solver, flags, cap=None):
    """On-device adaptation of a solver's mesh (dvm_adapt_*): flags (int8 per
    cell: +1 refine, -1 coarsen a complete sibling set, 0 keep) -> the new
    2:1-balanced leaf list (device), a solver on it with the same parameters,
    its face tables built on the device and its state remapped from `solver`.
    Returns (forest, mesh, solver)."""
    import dataclasses
    import torch
    n = solver.n
    cap = 8 * n if cap is None else int(cap)
    fl = torch.as_tensor(np.ascontiguousarray(flags, np.int8)).to("cuda")
    nb = C.c_size_t(0)
    _check(lib().dvm_adapt_workspace_bytes(cap + n, C.byref(nb)), "dvm_adapt_workspace_bytes")
    ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device="cuda")
    lev = torch.empty(cap, dtype=torch.uint8, device="cuda")
    ijk = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
    n_out = C.c_int64(0)
    _check(lib().dvm_adapt_leaves(solver.h, fl.data_ptr(), cap, lev.data_ptr(), ijk.data_ptr(), C.byref(n_out),
                                  ws.data_ptr(), nb.value, solver.stream()), "dvm_adapt_leaves")
    m = n_out.value
    mh = C.c_void_p()
    _check(lib().dvm_adapt_mesh(solver.mesh.h, lev.data_ptr(), ijk.data_ptr(), m, C.byref(mh), solver.stream()),
           "dvm_adapt_mesh")
    forest = dataclasses.replace(solver.mesh.forest, level=lev[:m].cpu().numpy(), ijk=ijk[:m].cpu().numpy())
    mesh = Mesh.wrap(mh, forest)
    new = Solver(mesh, solver.params)
    _check(lib().dvm_adapt_tables(new.h, lev.data_ptr(), ijk.data_ptr(), ws.data_ptr(), nb.value, new.stream()),
           "dvm_adapt_tables")
    mesh._info()  # face counts, known once the tables exist
    _check(lib().dvm_adapt_remap(solver.h, new.h, ws.data_ptr(), nb.value, new.stream()), "dvm_adapt_remap")
    return forest, mesh, new


class LBM:
    """The lattice Boltzmann subset (dvm_lbm_*): D3Q19 or D3Q27 on a mesh, torch buffers."""

    def __init__(self, mesh: Mesh, q=19, precision=PREC_FP32, tau=0.6, collision=COLL_EXP):
        import torch
        self.torch = torch
        self.mesh = mesh
        p = LbmParams(int(q), int(precision), int(collision), float(tau))
        h = C.c_void_p()
        _check(lib().dvm_lbm_create(mesh.h, C.byref(p), C.byref(h)), "dvm_lbm_create")
        self.h = h
        sz = Sizes()
        _check(lib().dvm_lbm_buffer_sizes(h, C.byref(sz)), "dvm_lbm_buffer_sizes")
        self.sizes = sz
        self.n, self.q = int(sz.n_cells), int(q)
        self.fdtype = torch.float64 if precision == PREC_FP64 else torch.float32

        def buf(nbytes):
            return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")

        self.f_a, self.f_b = buf(sz.f_bytes), buf(sz.f_bytes)
        self.mom = torch.empty((5, self.n), dtype=torch.float64, device="cuda")
        self.tables_buf = buf(sz.tables_bytes)
        self.ws = buf(sz.ws_bytes)
        _check(lib().dvm_lbm_bind(h, self.f_a.data_ptr(), self.f_b.data_ptr(), self.mom.data_ptr(),
                                  self.tables_buf.data_ptr(), self.ws.data_ptr()), "dvm_lbm_bind")
        _check(lib().dvm_lbm_upload(h, self.stream()), "dvm_lbm_upload")

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def init(self, prim):
        """f := f_eq of prim [4][n] (rho, ux, uy, uz)"""
        t = self.torch.as_tensor(np.ascontiguousarray(prim, np.float64)).to("cuda")
        self._prim = t
        _check(lib().dvm_lbm_init(self.h, t.data_ptr(), self.stream()), "dvm_lbm_init")

    def dt(self, cfl):
        out = C.c_double()
        _check(lib().dvm_lbm_dt(self.h, float(cfl), C.byref(out)), "dvm_lbm_dt")
        return out.value

    def step(self, n=1, dt=0.0, cfl=0.5):
        _check(lib().dvm_lbm_step(self.h, int(n), float(dt), float(cfl), self.stream()), "dvm_lbm_step")

    def moments(self):
        out = self.torch.empty((5, self.n), dtype=self.torch.float64, device="cuda")
        _check(lib().dvm_lbm_moments(self.h, out.data_ptr(), self.stream()), "dvm_lbm_moments")
        return out

    def check(self):
        d = Diag()
        rc = lib().dvm_lbm_check(self.h, self.stream(), C.byref(d))
        if rc not in (OK, ERR_NONPHYSICAL):
            _check(rc, "dvm_lbm_check")
        return rc, np.array(d.sums[:]), bool(d.nonphysical), int(d.steps)

    def f_canonical(self):
        out = self.torch.empty((self.n, 27), dtype=self.fdtype, device="cuda")
        _check(lib().dvm_lbm_get_f(self.h, out.data_ptr(), self.stream()), "dvm_lbm_get_f")
        return out

    def set_f_canonical(self, f):
        t = self.torch.as_tensor(np.ascontiguousarray(f)).to(device="cuda", dtype=self.fdtype)
        _check(lib().dvm_lbm_set_f(self.h, t.data_ptr(), self.stream()), "dvm_lbm_set_f")
        self.torch.cuda.synchronize()

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().dvm_destroy_lbm(self.h)
                self.h = None
        except Exception:
            pass


class Batch:
    """Many solvers advanced by one graph launch per step (dvm_batch_*)."""

    def __init__(self, solvers, cfl=0.5):
        import torch
        self.torch = torch
        self.solvers = list(solvers)  # keep them alive
        arr = (C.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = C.c_void_p()
        _check(lib().dvm_batch_create(arr, len(self.solvers), float(cfl), C.byref(h)), "dvm_batch_create")
        self.h = h
        nb = C.c_size_t(0)
        _check(lib().dvm_batch_workspace_bytes(h, C.byref(nb)), "dvm_batch_workspace_bytes")
        self.ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device="cuda")
        _check(lib().dvm_batch_bind(h, self.ws.data_ptr()), "dvm_batch_bind")

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def step(self, n=1):
        _check(lib().dvm_batch_step(self.h, int(n), self.stream()), "dvm_batch_step")

    def tune(self, reps=3, cache_path=None):
        """per-group kernel shapes by timing (dvm_batch_tune); groups found in
        the tuner cache file take the stored shape"""
        cp = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().dvm_batch_tune(self.h, int(reps), cp, self.stream()), "dvm_batch_tune")

    def branches(self, enable=-1):
        """groups as parallel graph branches (1) or one chain (0); -1 queries"""
        prev = C.c_int32(0)
        _check(lib().dvm_batch_branches(self.h, int(enable), C.byref(prev)), "dvm_batch_branches")
        return prev.value

    def groups(self):
        n = C.c_int32(0)
        _check(lib().dvm_batch_info(self.h, -1, None, C.byref(n), None, None, None, None, None, None),
               "dvm_batch_info")
        out = []
        for g in range(n.value):
            v = [C.c_int32(0) for _ in range(7)]
            cells = C.c_int64(0)
            ms = C.c_double(0)
            _check(lib().dvm_batch_info(self.h, g, C.byref(v[0]), C.byref(v[1]), C.byref(cells), C.byref(v[2]),
                                        C.byref(v[3]), C.byref(v[4]), C.byref(v[5]), C.byref(ms)), "dvm_batch_info")
            out.append(dict(nh=v[0].value, instances=v[1].value, cells=cells.value, threads=v[2].value,
                            wpe=v[3].value, xcd_group=v[4].value, nt_store=v[5].value, tuned_ms=ms.value))
        return out

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().dvm_destroy_batch(self.h)
                self.h = None
        except Exception:
            pass


def mlp_gradient_noalloc(params, x, y, pos_weight=1.0, grad=None, loss=None):
    """loss and weight gradients of the network with the library's static
    scratch (dvm_mlp_gradient_noalloc): no network object, no workspace.
    params, x, y, grad (float32 [MLP_WEIGHTS]) and loss (float64 [1]) are
    CUDA tensors; returns (grad, loss)."""
    import torch
    x, y = x.contiguous(), y.contiguous()
    if grad is None:
        grad = torch.empty(MLP_WEIGHTS, dtype=torch.float32, device="cuda")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
    _check(lib().dvm_mlp_gradient_noalloc(params.data_ptr(), x.data_ptr(), y.data_ptr(), x.shape[0],
                                          float(pos_weight), grad.data_ptr(), loss.data_ptr(),
                                          C.c_void_p(torch.cuda.current_stream().cuda_stream)),
           "dvm_mlp_gradient_noalloc")
    return grad, loss


class MLP:
    """The sensor network: parameters (torch float32 [MLP_PARAMS]) and the
    training workspace (dvm_mlp_*)."""

    def __init__(self, params, max_batch=4096):
        import torch
        self.torch = torch
        self.params = torch.as_tensor(np.ascontiguousarray(params, np.float32)).to("cuda").contiguous()
        assert self.params.numel() == MLP_PARAMS
        h = C.c_void_p()
        _check(lib().dvm_mlp_create(int(max_batch), C.byref(h)), "dvm_mlp_create")
        self.h = h
        nb = C.c_size_t(0)
        _check(lib().dvm_mlp_workspace_bytes(h, C.byref(nb)), "dvm_mlp_workspace_bytes")
        self.ws = torch.zeros(int(nb.value), dtype=torch.uint8, device="cuda")
        _check(lib().dvm_mlp_bind(h, self.params.data_ptr(), self.ws.data_ptr()), "dvm_mlp_bind")

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def set_normalization(self, x):
        x = x.contiguous()
        _check(lib().dvm_mlp_set_normalization(self.h, x.data_ptr(), x.shape[0], self.stream()),
               "dvm_mlp_set_normalization")

    def forward(self, x, mode=1):
        x = x.contiguous()
        z = self.torch.empty(x.shape[0], dtype=self.torch.float32, device="cuda")
        _check(lib().dvm_mlp_forward(self.h, x.data_ptr(), x.shape[0], int(mode), z.data_ptr(), self.stream()),
               "dvm_mlp_forward")
        return z

    def gradient(self, x, y, pos_weight=1.0):
        x, y = x.contiguous(), y.contiguous()
        _check(lib().dvm_mlp_gradient(self.h, x.data_ptr(), y.data_ptr(), x.shape[0], float(pos_weight),
                                      self.stream()), "dvm_mlp_gradient")

    def adam(self, lr):
        _check(lib().dvm_mlp_adam(self.h, float(lr), self.stream()), "dvm_mlp_adam")

    def train_step(self, x, y, lr, pos_weight=1.0):
        x, y = x.contiguous(), y.contiguous()
        _check(lib().dvm_mlp_train_step(self.h, x.data_ptr(), y.data_ptr(), x.shape[0], float(lr),
                                        float(pos_weight), self.stream()), "dvm_mlp_train_step")

    def grads_and_loss(self):
        """(gradient float32 [MLP_WEIGHTS], loss) of the last gradient call (synchronises)"""
        g, l = C.c_void_p(), C.c_void_p()
        _check(lib().dvm_mlp_buffers(self.h, C.byref(g), C.byref(l)), "dvm_mlp_buffers")
        self.torch.cuda.synchronize()
        base = self.ws.data_ptr()
        go, lo = g.value - base, l.value - base
        grads = self.ws[go:go + 4 * MLP_WEIGHTS].view(self.torch.float32).clone()
        loss = float(self.ws[lo:lo + 8].view(self.torch.float64).item())
        return grads, loss

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().dvm_destroy_mlp(self.h)
                self.h = None
        except Exception:
            pass
