"""De Vahl Davis natural convection (Section 4.1) on the GPU stepper.

The unit square, left wall cold (T_C = -0.5), right wall hot (T_H = 0.5),
top and bottom adiabatic, no-slip everywhere, v = T = 0 at t = 0, T_ref = 0.
Three discretisations of the same box: "hybrid" (two diagonal quarters
scattered, two regular), "regular" and "scattered".  The run reports the
average Nusselt number along the cold wall (Eq. (5): L/(T_H - T_C) times the
mean |dT/dn| over the cold-wall nodes) as it evolves to t_end, the vertical
velocity near the horizontal midline |y - 0.5| <= h (the section of Fig. 6),
and the wall-clock time of the stepping.

Usage:
    python -m paper_2303_01760_amd.dvd --h 0.01 --layout hybrid regular scattered --t-end 0.15
    python -m paper_2303_01760_amd.dvd --h 0.02 --layout horizontal vertical --delta-h 5 10 25 40
(the split layouts are the study of the scattered layer width delta_h).

Every step runs in the library's kernels; the host only averages |dT/dn|
over the cold-wall nodes at report times.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import hsm
from . import nodegen as ng


def cold_wall_nodes(q: ng.NodeSet) -> np.ndarray:
    """Nodes of the x = 0 face (group 0)."""
    return np.nonzero(q.group == 0)[0]


def nusselt(st: hsm.Stencils, T: torch.Tensor, nodes: np.ndarray, L: float = 1.0, dT: float = 1.0) -> float:
    """Eq. (5) averaged over `nodes`: the normal derivative comes from the
    library's operator application on T (caller order)."""
    Ti = st.to_internal(T.contiguous())
    dn = st.to_caller(st.apply(Ti, hsm.OP_DN)[0].contiguous())
    g = dn.cpu().numpy()[nodes]
    return float(L / dT * np.mean(np.abs(g)))


def run_case(q: ng.NodeSet, *, Ra: float, Pr: float = 0.71, T_ref: float, t_end: float, dt: float,
             cold: np.ndarray, m: int = 2, tol: float = 1e-10, reports: int = 30, max_steps: int | None = None,
             progress=None, label: str = "", checkpoint: str | None = None, budget_s: float | None = None) -> dict:
    """Step a node set from v = 0, T = its Dirichlet values (0 elsewhere) to
    t_end (or max_steps); return the history of Nu over the `cold` nodes.
    checkpoint: a .npz file holding v, T, p, the step count and the history
    so far: the run continues from it if it exists, and rewrites it at every
    report; budget_s: stop at the first report after this much stepping time
    (the result then has complete = False)."""
    nsteps = int(math.ceil(t_end / dt - 1e-9))
    if max_steps is not None:
        nsteps = min(nsteps, max_steps)
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    st = hsm.build_stencils(torch.tensor(q.x, device=dev), torch.tensor(q.kind, device=dev),
                            torch.tensor(q.normal, device=dev), q.h, m)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    v0 = torch.zeros((q.d, q.n), dtype=torch.float64, device=dev)
    T0 = torch.tensor(np.where(q.kind == ng.KIND_DIRICHLET, q.tbc, 0.0), device=dev)
    p0 = None
    hist = []
    done, t_step, iters_before = 0, 0.0, 0
    if checkpoint and os.path.exists(checkpoint):
        ck = np.load(checkpoint)
        if int(ck["n"]) != q.n or float(ck["dt"]) != dt:
            raise ValueError(f"checkpoint {checkpoint} is for another node set or time step")
        v0, T0, p0 = (torch.tensor(ck["v"], device=dev), torch.tensor(ck["T"], device=dev),
                      torch.tensor(ck["p"], device=dev))
        done, t_step, iters_before = int(ck["done"]), float(ck["stepping_s"]), int(ck["krylov_iters"])
        hist = [tuple(r) for r in ck["hist"].tolist()]
    sim = hsm.Sim(st, v0, T0, p0, Ra=Ra, Pr=Pr, dt=dt, T_ref=T_ref, krylov_tol=tol)
    per = max(1, nsteps // reports)
    t_run = 0.0
    while done < nsteps:
        if budget_s is not None and t_run > budget_s:
            break
        k = min(per, nsteps - done)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        sim.step(k)
        torch.cuda.synchronize()
        t_step += time.perf_counter() - ts
        t_run += time.perf_counter() - ts
        done += k
        stats = sim.stats()
        if stats["status"] != 0:
            raise hsm.HsmError(stats["status"], f"stepping failed at step {done}", -1)
        v, T, p = sim.read()
        nu = nusselt(st, T, cold)
        hist.append((done * dt, nu))
        iters = iters_before + stats["krylov_iters_total"]
        if checkpoint:
            np.savez(checkpoint + ".tmp.npz", v=v.cpu().numpy(), T=T.cpu().numpy(), p=p.cpu().numpy(), done=done,
                     n=q.n, dt=dt, stepping_s=t_step, krylov_iters=iters, hist=np.array(hist))
            os.replace(checkpoint + ".tmp.npz", checkpoint)
        if progress:
            progress(f"{label}: t={done * dt:.5f} ({done}/{nsteps} steps) Nu={nu:.4f} "
                     f"krylov iters/step {iters / done:.1f}")
    v, T, p = [a.cpu().numpy() for a in sim.read()]
    stats = sim.stats()
    info = st.info()
    sim.close()
    st.close()
    return dict(N=q.n, n_regular=int(info["n_regular"]), n_scattered=int(info["n_scattered"]),
                n_scattered_fill=int(np.sum(q.origin == 2)), n_lattice=int(np.sum(q.origin == 0)), Ra=Ra, Pr=Pr,
                dt=dt, t_end=nsteps * dt, steps=done, complete=done >= nsteps, krylov_tol=tol,
                krylov_iters_total=iters_before + stats["krylov_iters_total"],
                nu_final=hist[-1][1] if hist else None, nu_history=hist,
                build_s=t_build, stepping_s=t_step, ms_per_step=1e3 * t_step / max(done, 1), v=v, T=T)


def run(h: float = 0.01, layout: str = "hybrid", Ra: float = 1e6, Pr: float = 0.71, t_end: float = 0.15,
        dt: float | None = None, m: int = 2, tol: float = 1e-10, reports: int = 30, seed: int = ng.SEED_BASE + 6,
        delta_h: float = 4.0, progress=None, checkpoint: str | None = None, budget_s: float | None = None) -> dict:
    """The cavity to t_end; layout hybrid / regular / scattered, or
    horizontal / vertical (the split at h*delta_h); returns the Nu history
    and the midline profile."""
    if layout in ("horizontal", "vertical"):
        q = ng.dvd2d_split(h, delta_h, layout, seed=seed)
    else:
        q = ng.dvd2d(h, layout, seed=seed)
    dt = 0.1 * h * h / 2 if dt is None else dt      # the paper's time-step rule
    r = run_case(q, Ra=Ra, Pr=Pr, T_ref=0.0, t_end=t_end, dt=dt, cold=cold_wall_nodes(q), m=m, tol=tol,
                 reports=reports, progress=progress, label=f"{layout} h={h}", checkpoint=checkpoint,
                 budget_s=budget_s)
    v = r.pop("v")
    r.pop("T")
    mid = np.nonzero(np.abs(q.x[1] - 0.5) <= h)[0]
    order = mid[np.argsort(q.x[0][mid])]
    r.update(layout=layout, h=h, delta_h=delta_h if layout in ("horizontal", "vertical") else None,
             midline=dict(x=q.x[0][order].tolist(), y=q.x[1][order].tolist(), v_y=v[1][order].tolist()))
    return r


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--h", type=float, default=0.01)
    ap.add_argument("--layout", nargs="+", default=["hybrid"],
                    choices=["hybrid", "regular", "scattered", "horizontal", "vertical"])
    ap.add_argument("--delta-h", type=float, nargs="+", default=[4.0],
                    help="split layouts: the scattered part ends at h*delta_h")
    ap.add_argument("--Ra", type=float, default=1e6)
    ap.add_argument("--t-end", type=float, default=0.15)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--reports", type=int, default=30)
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    ap.add_argument("--checkpoint", default=None,
                    help="directory of per-run .npz checkpoints: a run continues from its checkpoint and rewrites "
                         "it at every report")
    ap.add_argument("--budget-s", type=float, default=None, help="stop each run after this much stepping time")
    a = ap.parse_args(argv)
    res = []
    for lay in a.layout:
        for dh in (a.delta_h if lay in ("horizontal", "vertical") else [None]):
            ck = None
            if a.checkpoint:
                os.makedirs(a.checkpoint, exist_ok=True)
                ck = os.path.join(a.checkpoint, f"dvd_{lay}_h{a.h}_d{dh}_Ra{a.Ra:g}.npz")
            r = run(h=a.h, layout=lay, Ra=a.Ra, t_end=a.t_end, tol=a.tol, reports=a.reports,
                    delta_h=dh if dh is not None else 4.0,
                    progress=lambda s: print(s, file=sys.stderr, flush=True), checkpoint=ck, budget_s=a.budget_s)
            print(json.dumps({k: r[k] for k in ("layout", "h", "delta_h", "N", "steps", "complete", "nu_final",
                                                "stepping_s", "krylov_iters_total")}), flush=True)
            res.append(r)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
