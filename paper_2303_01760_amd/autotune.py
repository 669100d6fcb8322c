"""Autotuner of the library's layout and launch parameters, timed on the
kernels that take the time.

Parameters searched (every candidate gives the same results up to the order
of floating-point sums; the weights do not change at all):
  build:  tile_log2     tile edge (2^L search cells per axis) of the internal
                        node order inside each width bucket;
          solve_groups  RBF-FD local systems per wave64 (1, 2, 3 where they fit);
  Krylov: wide_lanes    one or several threads per node of the non-regular
                        (wide) stencils in the Krylov kernels (or the
                        library's automatic choice);
          xcd_order     each XCD takes one contiguous run of the Krylov kernels'
                        blocks (where the reduction kernels run), or
                        consecutive blocks go to consecutive XCDs;
          block_nodes   nodes (threads) per block of the node kernels;
          gather_chunk  stencil entries per gather round of the BiCGSTAB p/v
                        kernel (loads in flight against registers held);
          krylov_chunk  BiCGSTAB iterations per device-side batch between
                        convergence checks;
          reduce_mode   one domain only: the Krylov dot products reduced in
                        every block's prologue, or by the reduction kernels
                        (or the library's choice by grid size).

What is timed:
  solve_groups: the device time of the RBF-FD buckets' local solves (the
      stencil build's per-bucket events), median of three builds;
  everything else: the pressure solve, about 97 % of a time step: the
      stepper runs `steps` time steps with start/stop events around every
      Krylov batch, and the figure is batch time per matrix-vector node row
      (with many domains each domain stops on its own, so time per iteration
      would not compare candidates fairly).

Search: one parameter at a time from the library defaults, in the order
above; a candidate replaces the current value only when it is faster by more
than `margin` (differences inside the timing noise would otherwise pick at
random).  Choices are cached in a JSON file (HSM_AUTOTUNE_CACHE, default
~/.cache/hsm/autotune.json) under a key of the device architecture,
dimension, layout, the width buckets, field precision and log2 of the node
count.
"""
from __future__ import annotations

import json
import math
import os
import statistics
import time

import torch

from . import hsm

DEFAULTS = dict(tile_log2=0, solve_groups=0, block_nodes=256, gather_chunk=8, krylov_chunk=32, xcd_order=0,
                wide_lanes=0, reduce_mode=0)
LANE_CANDIDATES = (0, 1, 2)
TILE_CANDIDATES = {2: (2, 3, 4), 3: (1, 2, 3)}
DEFAULT_TILE = {2: 3, 3: 2}
BLOCK_CANDIDATES = (128, 256, 64, 512)
GATHER_CANDIDATES = (8, 6, 12, 4)
BATCH_CANDIDATES = (32, 16, 64)


def cache_path() -> str:
    return os.environ.get("HSM_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "hsm",
                                                             "autotune.json"))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def cache_key(st: hsm.Stencils, mode: int, field_dtype: int) -> str:
    info = st.info()
    widths = ",".join(f"{t}:{w}" for t, w, c in info["buckets"] if c > 0)
    return (f"{_arch()}|d={info['d']}|mode={mode}|buckets={widths}|dtype={field_dtype}|"
            f"log2N={int(round(math.log2(max(info['n_nodes'], 1))))}")


def _load_cache(path):
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return {}


def _store_cache(path, key, rec):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    c = _load_cache(path)
    c[key] = rec
    tmp = path + ".tmp"
    json.dump(c, open(tmp, "w"), indent=1)
    os.replace(tmp, path)


def _solve_ms(build) -> float:
    """Device ms of the RBF-FD buckets' local solves, median of three builds."""
    ts = []
    for _ in range(3):
        st = build()
        info = st.info()
        ts.append(sum(ms for (t, w, c), ms in zip(info["buckets"], info["bucket_solve_ms"]) if t != 0 and c > 0))
        st.close()
    return statistics.median(ts)


def _krylov_ns_per_row(st, sim_kw, knobs, steps) -> float:
    """Krylov batch time per matvec node row (ns) over `steps` time steps from the given state."""
    sim = hsm.Sim(st, sim_kw["v0"], sim_kw["T0"], Ra=sim_kw["Ra"], Pr=sim_kw["Pr"], dt=sim_kw["dt"],
                  T_ref=sim_kw["T_ref"], krylov_tol=sim_kw["tol"], krylov_maxiter=sim_kw.get("maxiter", 200000),
                  field_dtype=sim_kw.get("field_dtype", hsm.F64), profile=1, block_nodes=knobs["block_nodes"],
                  gather_chunk=knobs["gather_chunk"], krylov_chunk=knobs["krylov_chunk"],
                  xcd_order=knobs["xcd_order"], wide_lanes=knobs["wide_lanes"], reduce_mode=knobs["reduce_mode"])
    try:
        sim.step(steps)
        ms, n = sim.phase_times()["krylov_batch"]
        rows = sim.stats()["krylov_node_matvecs"]
    finally:
        sim.close()
    return ms * n * 1e6 / max(rows, 1)


def tune(x: torch.Tensor, kind: torch.Tensor, normal: torch.Tensor, h, m, sim_kw: dict, mode=hsm.MODE_HYBRID,
         domain_offsets=None, n=None, steps: int = 1, margin: float = 0.03, use_cache: bool = True,
         path: str | None = None, log=None) -> dict:
    """Pick the parameters for this node set.  sim_kw: Ra, Pr, dt, T_ref, tol, v0, T0 (device tensors, caller
    order) and optionally field_dtype, maxiter.  Returns dict(choice=..., timings=..., cached=bool, key=...)."""
    d = int(x.shape[0])
    path = path or cache_path()
    field_dtype = sim_kw.get("field_dtype", hsm.F64)
    say = log or (lambda *_: None)

    def build(knobs):
        return hsm.build_stencils(x, kind, normal, h, m, mode=mode, domain_offsets=domain_offsets, n=n,
                                  tile_log2=knobs["tile_log2"], solve_groups=knobs["solve_groups"])

    cur = dict(DEFAULTS, tile_log2=DEFAULT_TILE[d])
    st0 = build(cur)
    key = cache_key(st0, mode, field_dtype)
    st0.close()
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit and set(hit.get("choice", {})) == set(DEFAULTS):
            return dict(choice=hit["choice"], timings=hit.get("timings", {}), cached=True, key=key)
    t_start = time.perf_counter()
    timings = {}

    def pick(name, cands, cost):
        res = {}
        for c in cands:
            trial = dict(cur, **{name: c})
            res[c] = cost(trial)
            say(f"autotune {name}={c}: {res[c]:.4g}")
        base = res.get(cur[name])
        best = min(res, key=res.get)
        if base is None or res[best] < (1.0 - margin) * base:
            cur[name] = best
        timings[name] = {str(k): v for k, v in res.items()}

    # systems per wave of the RBF-FD solves (only where more than one fits)
    st1 = build(cur)
    st_info = st1.info()
    st1.close()
    sizes = [w + math.comb(_deg(w, d) + d, d) for t, w, c in st_info["buckets"] if t != 0 and c > 0]
    gmax = max([3 if S <= 21 else 2 if S <= 32 else 1 for S in sizes] or [1])
    if gmax > 1:
        pick("solve_groups", [0] + list(range(1, gmax)), lambda k: _solve_ms(lambda: build(k)))

    def kry(k):
        # the events bracket the Krylov batches only: graph instantiation on the first step is not timed
        st = build(k)
        try:
            return _krylov_ns_per_row(st, sim_kw, k, steps)
        finally:
            st.close()

    pick("wide_lanes", LANE_CANDIDATES, kry)
    pick("tile_log2", TILE_CANDIDATES[d], kry)
    pick("xcd_order", (0, 1), kry)
    pick("block_nodes", BLOCK_CANDIDATES, kry)
    pick("gather_chunk", GATHER_CANDIDATES, kry)
    pick("krylov_chunk", BATCH_CANDIDATES, kry)
    if domain_offsets is None or len(domain_offsets) == 2:   # several domains always use the reduction kernels
        pick("reduce_mode", (0, 1, 2), kry)
    rec = dict(choice=cur, timings=timings, key=key, tuning_s=time.perf_counter() - t_start,
               units=dict(solve_groups="ms of RBF-FD solves per build",
                          other="ns of Krylov batch time per matvec node row"))
    if use_cache:
        _store_cache(path, key, rec)
    rec["cached"] = False
    return rec


def _deg(width: int, d: int) -> int:
    """Monomial degree m of an RBF-FD bucket from its stencil size n = 2 C(m+d, m)."""
    for mm in range(1, 5):
        if 2 * math.comb(mm + d, mm) == width:
            return mm
    return 2
