"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds no arithmetic of the method: it draws random numbers and
evaluates geometric predicates to produce (a) leaf lists of a forest of octrees
(before 2:1 balancing, which both sides perform themselves), (b) solid flags
from a ball predicate, (c) initial macroscopic fields (rho, u, T) at leaf
centres, and (d) the workload descriptions (velocity grid, boundary kinds,
relaxation parameters) of the synthetic problems shaped like the paper's
(section 3.3: 24^3 velocities on ~1e4-1e5 cells; section 3.4: ~1e6 kinetic
cells with 24^3 velocities).

Boundary kinds are plain integers with the values the C interface documents:
PERIODIC 0, INFLOW 1, OUTFLOW 2, WALL 3, domain faces in order -x,+x,-y,+y,-z,+z.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

PERIODIC, INFLOW, OUTFLOW, WALL = 0, 1, 2, 3
SCHEME_UPWIND1, SCHEME_MUSCL = 0, 1
COLL_EXP, COLL_EULER, COLL_OFF, COLL_KOROBOV = 0, 1, 2, 3
TAU_CONST, TAU_HS = 0, 1
PREC_FP64, PREC_FP32 = 0, 1


@dataclasses.dataclass
class Forest:
    """A leaf list: leaf t is the cube (level[t], ijk[t]) of edge h0 / 2**level."""
    base: tuple
    h0: float
    bc: tuple
    level: np.ndarray          # uint8 [n]
    ijk: np.ndarray            # int32 [n, 3]
    solid: Optional[np.ndarray] = None  # uint8 [n] or None

    @property
    def n(self) -> int:
        return int(self.level.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    forest: Forest             # before balancing
    nv: tuple                  # velocity nodes per axis
    vlo: tuple
    vhi: tuple
    scheme: int
    collision: int
    tau_mode: int
    tau_or_kn: float
    cfl: float
    steps: int
    inflow: tuple = (1.0, 0.0, 0.0, 0.0, 1.0)   # rho, ux, uy, uz, T
    t_wall: float = 1.0
    fields: str = "uniform"    # name of the initial-field recipe
    field_args: dict = dataclasses.field(default_factory=dict)
    solid_ball: Optional[tuple] = None          # (cx, cy, cz, r, level) -> solid leaves
    korobov_p: int = 0                          # collision COLL_KOROBOV: lattice points per node


# ----------------------------------------------------------------------------
# leaf lists
# ----------------------------------------------------------------------------

def uniform_forest(base=(1, 1, 1), level=0, h0=1.0, bc=(PERIODIC,) * 6) -> Forest:
    nx, ny, nz = (b << level for b in base)
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    ijk = g.reshape(-1, 3).astype(np.int32)
    lev = np.full(ijk.shape[0], level, np.uint8)
    return Forest(tuple(base), float(h0), tuple(bc), lev, ijk)


def _children(level: np.ndarray, ijk: np.ndarray):
    c = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], np.int32)
    kids = (2 * ijk[:, None, :] + c[None, :, :]).reshape(-1, 3)
    return np.repeat(level + 1, 8).astype(np.uint8), kids.astype(np.int32)


def refine(forest: Forest, mask: np.ndarray) -> Forest:
    """Replace the leaves flagged in mask by their 8 children."""
    keep = ~mask
    cl, ck = _children(forest.level[mask], forest.ijk[mask])
    return Forest(forest.base, forest.h0, forest.bc,
                  np.concatenate([forest.level[keep], cl]),
                  np.concatenate([forest.ijk[keep], ck]))


def random_root_refinement(base=(64, 64, 64), frac=0.4, seed=3, h0=None, bc=(PERIODIC,) * 6) -> Forest:
    """round(frac * #roots) roots, chosen by a seeded permutation, refined once."""
    h0 = 1.0 / base[0] if h0 is None else h0
    f = uniform_forest(base, 0, h0, bc)
    n_ref = int(round(frac * f.n))
    rng = np.random.default_rng(seed)
    mask = np.zeros(f.n, bool)
    mask[rng.permutation(f.n)[:n_ref]] = True
    return refine(f, mask)


def random_forest(seed: int, base=(2, 2, 2), extra_levels=3, p=0.3, bc=(PERIODIC,) * 6) -> Forest:
    """Random refinement (not balanced) for brute-force mesh checks."""
    rng = np.random.default_rng(seed)
    f = uniform_forest(base, 0, 1.0 / base[0], bc)
    for _ in range(extra_levels):
        mask = rng.random(f.n) < p
        if not mask.any():
            mask[rng.integers(f.n)] = True
        f = refine(f, mask)
    return f


def leaf_centres(forest: Forest) -> np.ndarray:
    h = forest.h0 / (2.0 ** forest.level.astype(np.float64))
    return (forest.ijk.astype(np.float64) + 0.5) * h[:, None]


def _cube_meets_ball(level, ijk, h0, centre, r):
    """Closed cube meets closed ball: clamp the centre into the cube (dyadic)."""
    h = h0 / (2.0 ** level.astype(np.float64))
    lo = ijk.astype(np.float64) * h[:, None]
    hi = lo + h[:, None]
    c = np.asarray(centre, np.float64)
    p = np.clip(c[None, :], lo, hi)
    d2 = ((p - c[None, :]) ** 2).sum(1)
    return d2 <= r * r


def sphere_refinement(base=(32, 32, 32), levels=2, centre=(0.5, 0.5, 0.5), radius=0.2,
                      bc=(INFLOW, OUTFLOW, OUTFLOW, OUTFLOW, OUTFLOW, OUTFLOW)) -> Forest:
    """Refine `levels` times every leaf whose closed cube meets the closed ball
    of radius radius + h_finest (one finest cell of margin, so that every leaf
    touching a solid leaf is itself at the finest level)."""
    h0 = 1.0 / base[0]
    f = uniform_forest(base, 0, h0, bc)
    h_fin = h0 / 2 ** levels
    for lev in range(levels):
        mask = (f.level == lev) & _cube_meets_ball(f.level, f.ijk, h0, centre, radius + h_fin)
        f = refine(f, mask)
    return f


def solid_flags(forest: Forest, centre, radius, level) -> np.ndarray:
    """A leaf at `level` is solid iff its centre lies strictly inside the ball."""
    x = leaf_centres(forest)
    d2 = ((x - np.asarray(centre)[None, :]) ** 2).sum(1)
    return ((forest.level == level) & (d2 < radius * radius)).astype(np.uint8)


# ----------------------------------------------------------------------------
# initial fields, [5][n] = rho, ux, uy, uz, T at leaf centres
# ----------------------------------------------------------------------------

def fields(recipe: str, x: np.ndarray, **kw) -> np.ndarray:
    n = x.shape[0]
    out = np.zeros((5, n))
    if recipe == "uniform":
        rho, u, T = kw.get("rho", 1.0), kw.get("u", (0.0, 0.0, 0.0)), kw.get("T", 1.0)
        out[0] = rho
        out[1:4] = np.asarray(u)[:, None]
        out[4] = T
    elif recipe == "sine_rho":      # rho = 1 + a sin(2 pi x), u = 0, T = 1
        a = kw.get("a", 0.1)
        out[0] = 1.0 + a * np.sin(2 * math.pi * x[:, 0])
        out[4] = 1.0
    elif recipe == "sod_x":         # rho, T jump at x = 1/2
        left = x[:, 0] < 0.5
        out[0] = np.where(left, kw.get("rho_l", 1.0), kw.get("rho_r", 0.125))
        out[4] = np.where(left, kw.get("T_l", 1.0), kw.get("T_r", 0.8))
    elif recipe == "sines":         # base + a sin(2 pi k.x + phi) per variable
        rng = np.random.default_rng(kw["seed"])
        amin, amax = kw.get("amin", 0.05), kw.get("amax", 0.2)
        ks = kw.get("kset", (1, 2))
        base = (1.0, 0.0, 0.0, 0.0, 1.0)
        for v in range(5):
            a = rng.uniform(amin, amax)
            k = rng.choice(ks, size=3)
            phi = rng.uniform(0, 2 * math.pi)
            out[v] = base[v] + a * np.sin(2 * math.pi * (x @ k) + phi)
    elif recipe == "sensor_runs":   # rho, u_b, T = base + a sin(2 pi k.x + phi), a ~ U[0, amax], k in {0,1,2}^3 \ 0
        rng = np.random.default_rng(kw["seed"])
        amax = kw.get("amax", 0.3)
        base = (1.0, 0.0, 0.0, 0.0, 1.0)
        for v in range(5):
            a = rng.uniform(0.0, amax)
            k = np.zeros(3, np.int64)
            while not k.any():
                k = rng.integers(0, 3, size=3)
            phi = rng.uniform(0, 2 * math.pi)
            out[v] = base[v] + a * np.sin(2 * math.pi * (x @ k) + phi)
    else:
        raise ValueError(recipe)
    return out


def sensor_run_tau(seed: int, lo: float = 0.01, hi: float = 1.0) -> float:
    """Relaxation time of one sensor training run: log-uniform in [lo, hi]."""
    rng = np.random.default_rng([seed, 7])
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


MLP_IN, MLP_HIDDEN = 10, 64
# parameter block: w1[64][10], b1[64], w2[64][64], b2[64], w3[64], b3, mean[10], std[10]
MLP_WEIGHTS = MLP_HIDDEN * MLP_IN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1
MLP_PARAMS = MLP_WEIGHTS + 2 * MLP_IN


def mlp_init(seed: int = 0) -> np.ndarray:
    """Seeded initial parameters of the 10-64-64-1 sensor network (uniform
    Glorot bounds, zero biases, identity normalisation), float32 block."""
    rng = np.random.default_rng(seed)
    p = np.zeros(MLP_PARAMS, np.float32)
    o = 0
    for fan_in, fan_out in ((MLP_IN, MLP_HIDDEN), (MLP_HIDDEN, MLP_HIDDEN), (MLP_HIDDEN, 1)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        p[o:o + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out)
        o += fan_in * fan_out + fan_out  # biases stay 0
    p[MLP_WEIGHTS + MLP_IN:] = 1.0  # std
    return p


# ----------------------------------------------------------------------------
# workloads shaped like the paper's
# ----------------------------------------------------------------------------

def batch_workloads(seed: int = 4, count: int = 64, cells_lo: float = 4e3, cells_hi: float = 2e5,
                    grids=(12, 16, 24), vmax: float = 6.0, kn: float = 0.05) -> list:
    """Independent periodic instances of uneven size for batched stepping:
    target cell counts log-uniform in [cells_lo, cells_hi]; half uniform root
    lattices, half with a seeded fraction U[0.1, 0.5] of the roots refined
    once; root box nx = ny = round(cbrt(roots)), nz = round(roots / nx^2);
    a velocity grid drawn from `grids` on [-vmax, vmax]^3; sinusoidal
    perturbations of rho, u, T (amplitudes U[0.05, 0.2], wave vectors in
    {1, 2}^3); tau from Kn (hard sphere)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        target = math.exp(rng.uniform(math.log(cells_lo), math.log(cells_hi)))
        refined = rng.random() < 0.5
        frac = rng.uniform(0.1, 0.5) if refined else 0.0
        roots = target / (1.0 + 7.0 * frac)
        nx = max(1, int(round(roots ** (1.0 / 3.0))))
        nz = max(1, int(round(roots / (nx * nx))))
        nv = int(rng.choice(grids))
        fseed = int(rng.integers(0, 2 ** 31))
        base = (nx, nx, nz)
        forest = (random_root_refinement(base, frac, fseed) if refined else uniform_forest(base, 0, 1.0 / nx))
        out.append(Workload(f"batch{seed}_{i}", forest, (nv,) * 3, (-vmax,) * 3, (vmax,) * 3, SCHEME_UPWIND1,
                            COLL_EXP, TAU_HS, kn, 0.5, 10, fields="sines", field_args={"seed": fseed}))
    return out


def workload(name: str) -> Workload:
    if name == "uniform16_v8_fp64":
        # 16^3 periodic cells, 8^3 velocities on [-4.5, 4.5]^3, rho = 1 + 0.1 sin 2 pi x
        return Workload(name, uniform_forest((1, 1, 1), 4, 1.0), (8, 8, 8), (-4.5,) * 3, (4.5,) * 3,
                        SCHEME_UPWIND1, COLL_EXP, TAU_CONST, 0.1, 0.5, 20, fields="sine_rho",
                        field_args={"a": 0.1})
    if name == "korobov16_v8":
        # the C1 mesh and flow with the Boltzmann collision integral on 1021 Korobov nodes per velocity
        return Workload(name, uniform_forest((1, 1, 1), 4, 1.0), (8, 8, 8), (-4.5,) * 3, (4.5,) * 3,
                        SCHEME_UPWIND1, COLL_KOROBOV, TAU_CONST, 0.5, 0.5, 4, fields="sine_rho",
                        field_args={"a": 0.1}, korobov_p=1021)
    if name == "sphere32_v24_muscl":
        # 32^3 roots, two levels at a ball r = 0.2, Mach-2 inflow at x = 0
        u_in = 2.0 * math.sqrt(5.0 / 3.0)
        return Workload(name, sphere_refinement(), (24, 24, 24), (-6.0,) * 3, (6.0,) * 3,
                        SCHEME_MUSCL, COLL_EXP, TAU_HS, 0.05, 0.5, 50,
                        inflow=(1.0, u_in, 0.0, 0.0, 1.0), t_wall=1.0,
                        fields="uniform", field_args={"rho": 1.0, "u": (u_in, 0.0, 0.0), "T": 1.0},
                        solid_ball=(0.5, 0.5, 0.5, 0.2, 2))
    if name.startswith("octree64_v24"):
        # 64^3 roots, a seeded fraction refined once, periodic Sod-like jump along x
        frac = 0.2 if name.endswith("p20") else 0.4
        return Workload(name, random_root_refinement((64, 64, 64), frac, 3), (24, 24, 24), (-6.0,) * 3,
                        (6.0,) * 3, SCHEME_UPWIND1, COLL_EXP, TAU_HS, 0.01, 0.5, 10, fields="sod_x")
    if name.startswith("octree32_v24") or name.startswith("octree16_v24"):
        # the same construction on fewer roots (CPU-baseline and parity sizes)
        nb = 32 if name.startswith("octree32") else 16
        frac = 0.2 if name.endswith("p20") else 0.4
        return Workload(name, random_root_refinement((nb, nb, nb), frac, 3), (24, 24, 24), (-6.0,) * 3,
                        (6.0,) * 3, SCHEME_UPWIND1, COLL_EXP, TAU_HS, 0.01, 0.5, 10, fields="sod_x")
    raise KeyError(name)
