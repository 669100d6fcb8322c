"""Seeded synthetic node sets (input generation only).

This module places nodes; it computes nothing of the method itself (no
neighbour search, classification, weights or operators).  Tests, the bench
and the smoke check feed the same node sets to the FP64 CPU oracle and to the
GPU library, so it is kept apart from both.

The node sets follow the paper's recipe for a hybrid discretisation
(Section 2): a regular lattice, with lattice nodes removed in a band around
irregular boundaries, and the band refilled by a scattered Poisson-disk
placement (Bridson 2007, radius h, 30 candidates; the paper's own fill
algorithm is external to it).  Circles and spheres stand in for the paper's
duck-shaped obstacles (Section 4.2), whose geometry exists only as a figure.

Workloads (seeds are 2303017600 + the workload number):
  1. differentially heated cavity, h=0.02, scattered band 0.1 along the walls
     (left wall T=1, right wall T=0, top/bottom adiabatic)      ~2.6k nodes
  2. unit square minus 20 circles (r ~ U(0.02, 0.08)), h=0.002, band 0.05
     around the circles, box walls adiabatic, circles T=0/1       ~230k nodes
  4. unit cube minus 8 spheres (r ~ U(0.05, 0.15)), h=0.01, band 0.05  ~950k
  5. workload 2 at h=0.001                                        ~900k nodes
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhsm_nodegen.so")
_lib = None

KIND_INTERIOR, KIND_DIRICHLET, KIND_NEUMANN = 0, 1, 2
SEED_BASE = 2303017600


class _Params(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("n_obst", ctypes.c_int32),
        ("h", ctypes.c_double), ("wall_band", ctypes.c_double), ("obst_band", ctypes.c_double),
        ("rmin", ctypes.c_double), ("rmax", ctypes.c_double), ("gap", ctypes.c_double),
        ("wall_kind", ctypes.c_int32 * 6), ("wall_T", ctypes.c_double * 6),
        ("obst_T", ctypes.c_double * 2), ("obst_kind", ctypes.c_int32),
        ("n_candidates", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("quarters", ctypes.c_int32), ("split_axis", ctypes.c_int32), ("split_pos", ctypes.c_double),
        ("h_s", ctypes.c_double),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"node generator library not built: {_LIB_PATH} (run __graft_entry__.build())")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.ng_generate.restype = ctypes.c_void_p
        lib.ng_generate.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_int64)]
        lib.ng_copy.restype = None
        lib.ng_copy.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6
        lib.ng_obstacles.restype = ctypes.c_int32
        lib.ng_obstacles.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.ng_free.restype = None
        lib.ng_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class NodeSet:
    """A node set of one domain.  Arrays are numpy; positions are SoA [d][N]."""
    d: int
    h: float                      # regular lattice spacing h_r
    x: np.ndarray                 # float64 [d, N]
    kind: np.ndarray              # uint8 [N]: 0 interior, 1 Dirichlet-T, 2 Neumann-T
    normal: np.ndarray            # float64 [d, N], outward unit normal (0 inside)
    tbc: np.ndarray               # float64 [N], Dirichlet temperature (0 elsewhere)
    origin: np.ndarray            # int8 [N]: 0 lattice, 1 boundary, 2 scattered fill
    group: np.ndarray             # int32 [N]: -1 fluid, 0..5 box face, 6+i obstacle i
    obstacles: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[1])


def generate(d: int, h: float, *, wall_band: float = 0.0, obst_band: float = 0.0,
             n_obst: int = 0, rmin: float = 0.0, rmax: float = 0.0, gap: float = 4.0,
             wall_kind=None, wall_T=None, obst_T=(0.0, 1.0), obst_kind: int = KIND_DIRICHLET,
             n_candidates: int = 30, quarters: bool = False, split_axis: int = -1, split_pos: float = 0.0,
             h_s: float = 0.0, seed: int = SEED_BASE, name: str = "") -> NodeSet:
    lib = _load()
    p = _Params()
    p.d, p.n_obst, p.h = d, n_obst, h
    p.wall_band, p.obst_band, p.rmin, p.rmax, p.gap = wall_band, obst_band, rmin, rmax, gap
    wk = list(wall_kind) if wall_kind is not None else [KIND_NEUMANN] * 6
    wt = list(wall_T) if wall_T is not None else [0.0] * 6
    for i in range(6):
        p.wall_kind[i] = int(wk[i]) if i < len(wk) else KIND_NEUMANN
        p.wall_T[i] = float(wt[i]) if i < len(wt) else 0.0
    p.obst_T[0], p.obst_T[1] = float(obst_T[0]), float(obst_T[1])
    p.obst_kind, p.n_candidates, p.seed = obst_kind, n_candidates, seed & 0xFFFFFFFFFFFFFFFF
    p.quarters, p.split_axis, p.split_pos, p.h_s = int(bool(quarters)), int(split_axis), float(split_pos), float(h_s)
    n = ctypes.c_int64(0)
    hnd = lib.ng_generate(ctypes.byref(p), ctypes.byref(n))
    if not hnd:
        raise ValueError("node generation failed (invalid parameters or obstacles could not be placed)")
    try:
        N = n.value
        x = np.empty((d, N), np.float64)
        kind = np.empty(N, np.uint8)
        nrm = np.empty((d, N), np.float64)
        tbc = np.empty(N, np.float64)
        origin = np.empty(N, np.int8)
        group = np.empty(N, np.int32)
        lib.ng_copy(hnd, x.ctypes.data, kind.ctypes.data, nrm.ctypes.data, tbc.ctypes.data,
                    origin.ctypes.data, group.ctypes.data)
        nob = lib.ng_obstacles(hnd, None)
        obst = np.zeros((nob, d + 1), np.float64)
        if nob:
            lib.ng_obstacles(hnd, obst.ctypes.data)
    finally:
        lib.ng_free(hnd)
    return NodeSet(d=d, h=h, x=x, kind=kind, normal=nrm, tbc=tbc, origin=origin, group=group,
                   obstacles=obst, name=name)


def cavity2d(h: float = 0.02, wall_band: float = 0.1, seed: int = SEED_BASE + 1,
             T_hot: float = 1.0, T_cold: float = 0.0) -> NodeSet:
    """Differentially heated cavity: left wall hot, right wall cold, top/bottom adiabatic."""
    return generate(2, h, wall_band=wall_band,
                    wall_kind=[KIND_DIRICHLET, KIND_DIRICHLET, KIND_NEUMANN, KIND_NEUMANN],
                    wall_T=[T_hot, T_cold, 0.0, 0.0], seed=seed, name=f"cavity2d_h{h}")


def dvd2d(h: float = 0.01, layout: str = "hybrid", seed: int = SEED_BASE + 6,
          T_cold: float = -0.5, T_hot: float = 0.5) -> NodeSet:
    """De Vahl Davis cavity (Section 4.1): left wall cold, right wall hot,
    top/bottom adiabatic.  layout "hybrid": the quarters x<1/2,y<1/2 and
    x>1/2,y>1/2 scattered, the other two a regular lattice; "regular": the
    lattice everywhere; "scattered": Poisson-disk nodes everywhere."""
    kinds = [KIND_DIRICHLET, KIND_DIRICHLET, KIND_NEUMANN, KIND_NEUMANN]
    temps = [T_cold, T_hot, 0.0, 0.0]
    if layout == "hybrid":
        return generate(2, h, quarters=True, wall_kind=kinds, wall_T=temps, seed=seed, name=f"dvd_hybrid_h{h}")
    if layout == "regular":
        return generate(2, h, wall_kind=kinds, wall_T=temps, seed=seed, name=f"dvd_regular_h{h}")
    if layout == "scattered":
        return generate(2, h, wall_band=0.6, wall_kind=kinds, wall_T=temps, seed=seed, name=f"dvd_scattered_h{h}")
    raise ValueError(f"unknown layout {layout!r}")


def dvd2d_split(h: float = 0.01, delta_h: float = 4.0, split: str = "horizontal", seed: int = SEED_BASE + 6,
                T_cold: float = -0.5, T_hot: float = 0.5) -> NodeSet:
    """The de Vahl Davis box split at distance h*delta_h from the origin
    (Section 4.1, the scattered-layer-width study): "horizontal" puts scattered
    nodes below y = h*delta_h and the lattice above, "vertical" scattered nodes
    left of x = h*delta_h.  delta_h = 0 is all lattice, h*delta_h >= 1 all
    scattered."""
    axis = {"vertical": 0, "horizontal": 1}[split]
    kinds = [KIND_DIRICHLET, KIND_DIRICHLET, KIND_NEUMANN, KIND_NEUMANN]
    temps = [T_cold, T_hot, 0.0, 0.0]
    return generate(2, h, split_axis=axis, split_pos=h * delta_h, wall_kind=kinds, wall_T=temps, seed=seed,
                    name=f"dvd_{split}_h{h}_d{delta_h}")


def refined2d(h_r: float = 0.01, ratio: float = 3.0, delta_h: float = 4.0, n_obst: int = 4,
              rmin: float = 0.05, rmax: float = 0.1, scattered: bool = False,
              seed: int = SEED_BASE + 7) -> NodeSet:
    """Irregular 2D domain with h-refinement (Section 4.2): the unit square
    minus n_obst circles (standing in for the duck shapes), spacing h_r/ratio
    on the circles growing linearly to h_r over h_r*delta_h, which is also the
    width of the scattered layer; scattered=True fills the whole box (same
    refinement).  Box walls adiabatic, circles alternately T=0 / T=1."""
    band = h_r * delta_h
    return generate(2, h_r, obst_band=band, wall_band=0.6 if scattered else 0.0, n_obst=n_obst, rmin=rmin,
                    rmax=rmax, h_s=h_r / ratio, wall_kind=[KIND_NEUMANN] * 4, seed=seed,
                    name=f"refined2d_h{h_r}_d{delta_h}{'_scattered' if scattered else ''}")


def refined3d(h_r: float = 0.025, ratio: float = 2.0, delta_h: float = 4.0, n_obst: int = 4,
              rmin: float = 0.08, rmax: float = 0.15, scattered: bool = False,
              seed: int = SEED_BASE + 8) -> NodeSet:
    """The paper's 3D case (Section 4.3): the unit cube minus n_obst spheres,
    spacing h_r/ratio on the spheres growing linearly to h_r over h_r*delta_h;
    box walls adiabatic, spheres alternately T=0 / T=1."""
    band = h_r * delta_h
    return generate(3, h_r, obst_band=band, wall_band=0.6 if scattered else 0.0, n_obst=n_obst, rmin=rmin,
                    rmax=rmax, h_s=h_r / ratio, wall_kind=[KIND_NEUMANN] * 6, seed=seed,
                    name=f"refined3d_h{h_r}_d{delta_h}{'_scattered' if scattered else ''}")


def obstacles2d(h: float = 0.002, n_obst: int = 20, rmin: float = 0.02, rmax: float = 0.08,
                band: float = 0.05, seed: int = SEED_BASE + 2) -> NodeSet:
    """Unit square minus seeded circles; adiabatic box, circles alternately T=0 / T=1."""
    return generate(2, h, obst_band=band, n_obst=n_obst, rmin=rmin, rmax=rmax,
                    wall_kind=[KIND_NEUMANN] * 4, seed=seed, name=f"obstacles2d_h{h}_n{n_obst}")


def obstacles3d(h: float = 0.01, n_obst: int = 8, rmin: float = 0.05, rmax: float = 0.15,
                band: float = 0.05, seed: int = SEED_BASE + 4) -> NodeSet:
    """Unit cube minus seeded spheres; adiabatic box, spheres alternately T=0 / T=1."""
    return generate(3, h, obst_band=band, n_obst=n_obst, rmin=rmin, rmax=rmax,
                    wall_kind=[KIND_NEUMANN] * 6, seed=seed, name=f"obstacles3d_h{h}_n{n_obst}")


def random_cloud(n: int, d: int = 2, seed: int = 0, h: float = 0.1) -> NodeSet:
    """Uniform random interior points in the unit box (tests only; no boundary)."""
    rng = np.random.default_rng(seed)
    x = rng.random((d, n))
    z = np.zeros(n)
    return NodeSet(d=d, h=h, x=x, kind=np.zeros(n, np.uint8), normal=np.zeros((d, n)), tbc=z.copy(),
                   origin=np.full(n, 2, np.int8), group=np.full(n, -1, np.int32), name=f"cloud{d}d_{n}")


@dataclass
class Batch:
    """Independent domains concatenated: domain k holds nodes [off[k], off[k+1])."""
    d: int
    x: np.ndarray                 # float64 [d, N]
    kind: np.ndarray              # uint8 [N]
    normal: np.ndarray            # float64 [d, N]
    tbc: np.ndarray               # float64 [N]
    off: np.ndarray               # int64 [K+1]
    h: np.ndarray                 # float64 [K], lattice spacing per domain
    m: np.ndarray                 # int32 [K], scattered polynomial degree per domain
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_domains(self) -> int:
        return len(self.off) - 1


def batch2d(n_domains: int = 512, nmin: int = 1000, nmax: int = 50000, n_obst: int = 4,
            seed_base: int = SEED_BASE * 10) -> Batch:
    """Many independent 2D obstacle domains of uneven size: domain k draws, from
    seed seed_base + k, a node count log-uniform in [nmin, nmax] (which sets its
    lattice spacing h = 1/round(sqrt(count / 0.8))), a scattered degree m in
    {2, 4}, and n_obst circles of radius max(0.04, 3.5h) to max(0.1, 5h) with a
    band max(0.05, 3h).  Every circle spans at least 3.5 node spacings in
    radius: circles of 1.6h make the explicit projection grow without bound
    (with m = 2 and m = 4 alike), circles of 3h stay stable.  Where n_obst such
    circles do not fit, the domain takes one fewer until they do."""
    sets, hs, ms = [], [], []
    for k in range(n_domains):
        rng = np.random.default_rng(seed_base + k)
        target = float(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
        m = int(rng.choice([2, 4]))
        h = 1.0 / max(8, int(round(np.sqrt(target / 0.8))))   # the lattice must divide the unit box
        band = max(0.05, 3.0 * h)
        s = None
        for no in range(n_obst, 0, -1):
            try:
                s = generate(2, h, obst_band=band, n_obst=no, rmin=max(0.04, 3.5 * h), rmax=max(0.1, 5.0 * h),
                             wall_kind=[KIND_NEUMANN] * 4, seed=seed_base + k, name=f"batch_{k}")
                break
            except ValueError:
                if no == 1:
                    raise
        sets.append(s)
        hs.append(h)
        ms.append(m)
    off = np.cumsum([0] + [s.n for s in sets]).astype(np.int64)
    return Batch(d=2, x=np.concatenate([s.x for s in sets], axis=1), kind=np.concatenate([s.kind for s in sets]),
                 normal=np.concatenate([s.normal for s in sets], axis=1), tbc=np.concatenate([s.tbc for s in sets]),
                 off=off, h=np.asarray(hs), m=np.asarray(ms, np.int32), name=f"batch2d_{n_domains}")
