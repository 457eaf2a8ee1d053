"""Python side of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It loads oracle/liboracle.so (plain C, FP64, OpenMP; see
dvm_oracle.c) and adds pure-Python brute-force checks for tiny meshes.
Nothing here is shared with, or imported by, the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

FACE_SAME, FACE_COARSER, FACE_FINER, FACE_INFLOW, FACE_OUTFLOW, FACE_WALL = range(6)


class OrParams(C.Structure):
    _fields_ = [("nv", C.c_int * 3), ("vlo", C.c_double * 3), ("vhi", C.c_double * 3),
                ("scheme", C.c_int), ("collision", C.c_int), ("tau_mode", C.c_int),
                ("tau_or_kn", C.c_double), ("inflow", C.c_double * 5), ("t_wall", C.c_double),
                ("korobov_p", C.c_int64), ("korobov_a", C.c_int64), ("lbm_q", C.c_int)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401  (python oracle/build.py)
            _b.build()
        L = C.CDLL(path)
        P = C.c_void_p
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        L.or_balance.argtypes = [i32p, i32p, C.c_int64, u8p, i32p, C.c_int64, C.POINTER(C.c_int64), u8p, i32p]
        L.or_mesh_new.argtypes = [i32p, C.c_double, i32p, C.c_int64, u8p, i32p, P, C.POINTER(P)]
        L.or_mesh_free.argtypes = [P]
        L.or_mesh_n_cells.argtypes = [P]
        L.or_mesh_n_cells.restype = C.c_int64
        L.or_mesh_n_leaves.argtypes = [P]
        L.or_mesh_n_leaves.restype = C.c_int64
        L.or_mesh_export.argtypes = [P, u64p, i64p, u8p, i32p, u8p, i32p]
        L.or_solver_new.argtypes = [P, C.POINTER(OrParams), C.POINTER(P)]
        L.or_solver_new_subset.argtypes = [P, C.POINTER(OrParams), C.c_int64, P, C.POINTER(P)]
        L.or_solver_rows.argtypes = [P]
        L.or_solver_rows.restype = C.c_int64
        L.or_valid.argtypes = [P, u8p]
        L.or_solver_free.argtypes = [P]
        L.or_solver_nv.argtypes = [P]
        L.or_solver_nv.restype = C.c_int64
        L.or_set_f.argtypes = [P, f64p]
        L.or_get_f.argtypes = [P, f64p]
        L.or_flag.argtypes = [P]
        L.or_init_maxwellian.argtypes = [P, f64p]
        L.or_init_lbm.argtypes = [P, f64p]
        L.or_step.argtypes = [P, C.c_double, C.c_int]
        L.or_transport.argtypes = [P, C.c_double]
        L.or_moments.argtypes = [P, f64p]
        L.or_global_sums.argtypes = [P, f64p]
        L.or_dt_cfl.argtypes = [P, C.c_double]
        L.or_dt_cfl.restype = C.c_double
        L.or_cell_maxwellian.argtypes = [i32p, f64p, f64p, f64p, f64p]
        L.or_cell_moments.argtypes = [i32p, f64p, f64p, f64p, f64p]
        L.or_cell_collide.argtypes = [C.POINTER(OrParams), C.c_double, f64p, f64p]
        L.or_korobov_generator.argtypes = [C.c_int64]
        L.or_korobov_generator.restype = C.c_int64
        L.or_korobov_tables.argtypes = [i32p, f64p, f64p, C.c_int64, C.c_int64, P, P, P, P]
        L.or_korobov_cell.argtypes = [i32p, f64p, f64p, C.c_int64, C.c_int64, f64p, f64p, f64p, f64p]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        _LIB = L
    return _LIB


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, np.int32))


def balance(forest):
    """Oracle 2:1 balance; returns (level u8[n], ijk i32[n,3]) in Morton order."""
    base = _i32(forest.base)
    per = _i32([forest.bc[2 * a] == 0 for a in range(3)])
    lev = np.ascontiguousarray(forest.level, np.uint8)
    ijk = np.ascontiguousarray(forest.ijk, np.int32).reshape(-1)
    cap = C.c_int64(0)
    n_out = C.c_int64(0)
    rc = lib().or_balance(base, per, forest.n, lev, ijk, 0, C.byref(n_out), np.zeros(1, np.uint8),
                          np.zeros(3, np.int32))
    if rc not in (0, -1):
        raise RuntimeError(f"or_balance: {rc}")
    cap = n_out.value
    lo = np.zeros(cap, np.uint8)
    io = np.zeros(3 * cap, np.int32)
    rc = lib().or_balance(base, per, forest.n, lev, ijk, cap, C.byref(n_out), lo, io)
    if rc:
        raise RuntimeError(f"or_balance: {rc}")
    return lo, io.reshape(-1, 3)


class Mesh:
    def __init__(self, forest, solid: Optional[np.ndarray] = None):
        self.forest = forest
        h = C.c_void_p()
        sol = None if solid is None else np.ascontiguousarray(solid, np.uint8)
        self._solid = sol
        rc = lib().or_mesh_new(_i32(forest.base), forest.h0, _i32(forest.bc), forest.n,
                               np.ascontiguousarray(forest.level, np.uint8),
                               np.ascontiguousarray(forest.ijk, np.int32).reshape(-1),
                               None if sol is None else sol.ctypes.data_as(C.c_void_p), C.byref(h))
        self.rc = rc
        if rc:
            raise RuntimeError(f"or_mesh_new: {rc}")
        self.h = h
        self.n_cells = int(lib().or_mesh_n_cells(h))
        self.n_leaves = int(lib().or_mesh_n_leaves(h))

    def tables(self):
        n = self.n_cells
        key = np.zeros(n, np.uint64)
        inp = np.zeros(n, np.int64)
        lev = np.zeros(n, np.uint8)
        ijk = np.zeros(3 * n, np.int32)
        ty = np.zeros(6 * n, np.uint8)
        nb = np.zeros(24 * n, np.int32)
        lib().or_mesh_export(self.h, key, inp, lev, ijk, ty, nb)
        return dict(key=key, input=inp, level=lev, ijk=ijk.reshape(n, 3), type=ty.reshape(n, 6),
                    nbr=nb.reshape(n, 6, 4))

    def cone(self, cells, hops):
        """the cells within `hops` face-neighbour steps of `cells` (sorted):
        what the state of `cells` after `hops` transport steps depends on"""
        t = self.tables()
        ty, nb = t["type"], t["nbr"]
        seen = np.zeros(self.n_cells, bool)
        front = np.unique(np.asarray(cells, np.int64))
        seen[front] = True
        for _ in range(int(hops)):
            tf = ty[front]
            k = np.where(tf == FACE_FINER, 4, np.where((tf == FACE_SAME) | (tf == FACE_COARSER), 1, 0))
            nxt = np.unique(nb[front][np.arange(4)[None, None, :] < k[:, :, None]]).astype(np.int64)
            front = nxt[~seen[nxt]]
            seen[front] = True
        return np.nonzero(seen)[0].astype(np.int64)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_mesh_free(self.h)
            self.h = None


def make_params(nv, vlo, vhi, scheme=0, collision=0, tau_mode=0, tau_or_kn=0.1,
                inflow=(1.0, 0.0, 0.0, 0.0, 1.0), t_wall=1.0, korobov_p=0, korobov_a=0, lbm_q=0) -> OrParams:
    p = OrParams()
    for a in range(3):
        p.nv[a] = int(nv[a])
        p.vlo[a] = float(vlo[a])
        p.vhi[a] = float(vhi[a])
    p.scheme, p.collision, p.tau_mode = int(scheme), int(collision), int(tau_mode)
    p.tau_or_kn = float(tau_or_kn)
    for a in range(5):
        p.inflow[a] = float(inflow[a])
    p.t_wall = float(t_wall)
    p.korobov_p, p.korobov_a = int(korobov_p), int(korobov_a)
    p.lbm_q = int(lbm_q)
    return p


def lbm_params(q, tau, collision=4, scheme=0):
    """LBM on the octree: the D3Q19 / D3Q27 subset of the 3^3 grid on [-3/2, 3/2]^3"""
    return make_params((3, 3, 3), (-1.5,) * 3, (1.5,) * 3, scheme=scheme, collision=collision, tau_or_kn=tau,
                       lbm_q=q)


class Solver:
    """The oracle's state on every cell of the mesh, or (cells = ascending
    cell indices) only on those cells: then rows follow `cells`, and valid()
    tells which rows are still exact (each step loses the cells that read a
    neighbour not held or no longer exact)."""

    def __init__(self, mesh: Mesh, params: OrParams, cells=None):
        self.mesh = mesh
        self.params = params
        h = C.c_void_p()
        if cells is None:
            rc = lib().or_solver_new(mesh.h, C.byref(params), C.byref(h))
            self.cells = None
        else:
            self.cells = np.ascontiguousarray(cells, np.int64)
            rc = lib().or_solver_new_subset(mesh.h, C.byref(params), self.cells.shape[0],
                                            self.cells.ctypes.data_as(C.c_void_p), C.byref(h))
        if rc:
            raise RuntimeError(f"or_solver_new: {rc}")
        self.h = h
        self.nv = int(lib().or_solver_nv(h))
        self.n = int(lib().or_solver_rows(h))

    def valid(self):
        out = np.zeros(self.n, np.uint8)
        lib().or_valid(self.h, out)
        return out.astype(bool)

    def set_f(self, f):
        lib().or_set_f(self.h, np.ascontiguousarray(f, np.float64).reshape(-1))

    def get_f(self):
        out = np.zeros(self.n * self.nv)
        lib().or_get_f(self.h, out)
        return out.reshape(self.n, self.nv)

    def init_lbm(self, prim):
        """LBM: f := f_eq of (rho, ux, uy, uz) [4][n]"""
        rc = lib().or_init_lbm(self.h, np.ascontiguousarray(prim, np.float64).reshape(-1))
        if rc:
            raise RuntimeError(f"or_init_lbm: {rc}")

    def init_maxwellian(self, prim):
        rc = lib().or_init_maxwellian(self.h, np.ascontiguousarray(prim, np.float64).reshape(-1))
        if rc:
            raise RuntimeError(f"or_init_maxwellian: {rc}")

    def step(self, dt, n=1):
        return int(lib().or_step(self.h, float(dt), int(n)))

    def transport(self, dt):
        lib().or_transport(self.h, float(dt))

    def moments(self):
        out = np.zeros(5 * self.n)
        lib().or_moments(self.h, out)
        return out.reshape(5, self.n)

    def global_sums(self):
        out = np.zeros(5)
        lib().or_global_sums(self.h, out)
        return out

    def dt_cfl(self, cfl):
        return float(lib().or_dt_cfl(self.h, float(cfl)))

    def flag(self):
        return int(lib().or_flag(self.h))

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_solver_free(self.h)
            self.h = None


def korobov_generator(p):
    """Korobov's optimal 5-dimensional generator for a p-point lattice (P_2 criterion)"""
    return int(lib().or_korobov_generator(int(p)))


def korobov_tables(nv, vlo, vhi, p, a):
    """(j, l, m, W), each [N^3, p]: partner node, post-collision nodes (-1: off the grid), weight"""
    n = int(np.prod(nv)) * int(p)
    j, l, m = (np.zeros(n, np.int32) for _ in range(3))
    W = np.zeros(n)
    rc = lib().or_korobov_tables(np.asarray(nv, np.int32), np.asarray(vlo, np.float64), np.asarray(vhi, np.float64),
                                 int(p), int(a), j.ctypes.data, l.ctypes.data, m.ctypes.data, W.ctypes.data)
    if rc:
        raise RuntimeError(f"or_korobov_tables: {rc}")
    sh = (int(np.prod(nv)), int(p))
    return j.reshape(sh), l.reshape(sh), m.reshape(sh), W.reshape(sh)


def korobov_cell(nv, vlo, vhi, p, a, f):
    """(I, B, C) of one cell: eq. (6), (4), (5)"""
    n = int(np.prod(nv))
    f = np.ascontiguousarray(f, np.float64)
    I, B, Cc = np.zeros(n), np.zeros(n), np.zeros(n)
    rc = lib().or_korobov_cell(np.asarray(nv, np.int32), np.asarray(vlo, np.float64), np.asarray(vhi, np.float64),
                               int(p), int(a), f, I, B, Cc)
    if rc:
        raise RuntimeError(f"or_korobov_cell: {rc}")
    return I, B, Cc


def cell_maxwellian(nv, vlo, vhi, prim):
    n = int(np.prod(nv))
    out = np.zeros(n)
    rc = lib().or_cell_maxwellian(_i32(nv), np.asarray(vlo, np.float64), np.asarray(vhi, np.float64),
                                  np.asarray(prim, np.float64), out)
    if rc:
        raise RuntimeError(f"or_cell_maxwellian: {rc}")
    return out


def cell_moments(nv, vlo, vhi, f):
    out = np.zeros(5)
    lib().or_cell_moments(_i32(nv), np.asarray(vlo, np.float64), np.asarray(vhi, np.float64),
                          np.ascontiguousarray(f, np.float64), out)
    return out


def cell_collide(params: OrParams, dt, fs):
    out = np.zeros_like(np.asarray(fs, np.float64))
    rc = lib().or_cell_collide(C.byref(params), float(dt), np.ascontiguousarray(fs, np.float64), out)
    return rc, out


# ----------------------------------------------------------------------------
# brute force for tiny meshes (pure Python, O(n^2))
# ----------------------------------------------------------------------------

def _extent(level, ijk, finest):
    s = 1 << (finest - int(level))
    lo = [int(c) * s for c in ijk]
    return lo, s


def brute_is_balanced(forest) -> bool:
    """2:1 over faces, edges and corners, by checking every pair of leaves."""
    finest = int(forest.level.max())
    ext = [b << finest for b in forest.base]
    per = [forest.bc[2 * a] == 0 for a in range(3)]
    boxes = [_extent(l, c, finest) for l, c in zip(forest.level, forest.ijk)]
    n = forest.n
    for a in range(n):
        la, sa = boxes[a]
        for b in range(n):
            if a == b or abs(int(forest.level[a]) - int(forest.level[b])) < 2:
                continue
            lb, sb = boxes[b]
            if _touch(la, sa, lb, sb, ext, per):
                return False
    return True


def _touch(la, sa, lb, sb, ext, per):
    """closed boxes intersect (periodic images included)"""
    for ax in range(3):
        ok = False
        shifts = (0, -ext[ax], ext[ax]) if per[ax] else (0,)
        for sh in shifts:
            lo_b = lb[ax] + sh
            if la[ax] <= lo_b + sb and lo_b <= la[ax] + sa:
                ok = True
        if not ok:
            return False
    return True


def brute_faces(forest, solid=None):
    """Face tables by O(n^2) enumeration of shared face area between leaves.

    Returns (order, type[n,6], nbr[n,6,4]) for the fluid leaves in ascending
    Morton order, with the same conventions as the oracle: faces -x,+x,-y,+y,
    -z,+z; SAME/COARSER one neighbour, FINER four neighbours ascending by key;
    boundary kinds from forest.bc; fluid-solid faces WALL.
    """
    finest = int(forest.level.max())
    ext = [b << finest for b in forest.base]
    per = [forest.bc[2 * a] == 0 for a in range(3)]
    n = forest.n
    sol = np.zeros(n, np.uint8) if solid is None else np.asarray(solid, np.uint8)

    def key(t):
        lo, _ = _extent(forest.level[t], forest.ijk[t], finest)
        k = 0
        for b in range(21):
            for ax in range(3):
                k |= ((lo[ax] >> b) & 1) << (3 * b + ax)
        return k

    keys = [key(t) for t in range(n)]
    order_all = sorted(range(n), key=lambda t: keys[t])
    fluid = [t for t in order_all if not sol[t]]
    rank = {t: r for r, t in enumerate(fluid)}
    boxes = [_extent(l, c, finest) for l, c in zip(forest.level, forest.ijk)]
    nf = len(fluid)
    ty = np.zeros((nf, 6), np.uint8)
    nb = -np.ones((nf, 6, 4), np.int32)
    bc_kind = {1: FACE_INFLOW, 2: FACE_OUTFLOW, 3: FACE_WALL}
    for r, a in enumerate(fluid):
        la, sa = boxes[a]
        for f in range(6):
            ax, side = f // 2, f % 2
            plane = la[ax] + (sa if side else 0)
            if not per[ax] and (plane == 0 or plane == ext[ax]):
                ty[r, f] = bc_kind[forest.bc[f]]
                continue
            found = []
            for b in range(n):
                if b == a:
                    continue
                lb, sb = boxes[b]
                # b's opposite face must lie on the plane (mod the period)
                bplane = lb[ax] + (0 if side else sb)
                if per[ax]:
                    if (bplane - plane) % ext[ax]:
                        continue
                elif bplane != plane:
                    continue
                area = 1
                for t in range(3):
                    if t == ax:
                        continue
                    ov = min(la[t] + sa, lb[t] + sb) - max(la[t], lb[t])
                    if ov <= 0:
                        area = 0
                        break
                    area *= ov
                if area > 0:
                    found.append(b)
            if any(sol[b] for b in found):
                assert all(sol[b] for b in found)
                ty[r, f] = FACE_WALL
                continue
            if len(found) == 1:
                b = found[0]
                ty[r, f] = FACE_SAME if forest.level[b] == forest.level[a] else FACE_COARSER
                nb[r, f, 0] = rank[b]
            else:
                assert len(found) == 4, found
                ty[r, f] = FACE_FINER
                nb[r, f, :] = sorted(rank[b] for b in found)
    return np.array(fluid), ty, nb
