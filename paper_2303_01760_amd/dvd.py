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

Every step runs in the library's kernels; the host only averages |dT/dn|
over the cold-wall nodes at report times.
"""
from __future__ import annotations

import argparse
import json
import math
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


def run(h: float = 0.01, layout: str = "hybrid", Ra: float = 1e6, Pr: float = 0.71, t_end: float = 0.15,
        dt: float | None = None, m: int = 2, tol: float = 1e-10, reports: int = 30, seed: int = ng.SEED_BASE + 6,
        progress=None) -> dict:
    """Step the cavity to t_end; return the Nu history and the midline profile."""
    q = ng.dvd2d(h, layout, seed=seed)
    dt = 0.1 * h * h / 2 if dt is None else dt      # the paper's time-step rule
    nsteps = int(math.ceil(t_end / dt - 1e-9))
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    st = hsm.build_stencils(torch.tensor(q.x, device=dev), torch.tensor(q.kind, device=dev),
                            torch.tensor(q.normal, device=dev), h, m)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    v0 = torch.zeros((2, q.n), dtype=torch.float64, device=dev)
    T0 = torch.tensor(np.where(q.kind == ng.KIND_DIRICHLET, q.tbc, 0.0), device=dev)
    sim = hsm.Sim(st, v0, T0, Ra=Ra, Pr=Pr, dt=dt, T_ref=0.0, krylov_tol=tol)
    cold = cold_wall_nodes(q)
    hist = []
    done, t_step = 0, 0.0
    per = max(1, nsteps // reports)
    while done < nsteps:
        k = min(per, nsteps - done)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        sim.step(k)
        torch.cuda.synchronize()
        t_step += time.perf_counter() - ts
        done += k
        stats = sim.stats()
        if stats["status"] != 0:
            raise hsm.HsmError(stats["status"], f"stepping failed at step {done}", -1)
        _, T, _ = sim.read()
        nu = nusselt(st, T, cold)
        hist.append((done * dt, nu))
        if progress:
            progress(f"{layout} h={h}: t={done * dt:.4f} ({done}/{nsteps} steps) Nu={nu:.4f} "
                     f"krylov iters/step {stats['krylov_iters_total'] / done:.1f}")
    v, T, p = [a.cpu().numpy() for a in sim.read()]
    stats = sim.stats()
    mid = np.nonzero(np.abs(q.x[1] - 0.5) <= h)[0]
    order = mid[np.argsort(q.x[0][mid])]
    sim.close()
    st.close()
    return dict(layout=layout, h=h, N=q.n, n_scattered_fill=int(np.sum(q.origin == 2)),
                n_lattice=int(np.sum(q.origin == 0)), Ra=Ra, Pr=Pr, dt=dt, t_end=nsteps * dt, steps=nsteps,
                krylov_tol=tol, krylov_iters_total=stats["krylov_iters_total"],
                nu_final=hist[-1][1], nu_history=hist, build_s=t_build, stepping_s=t_step,
                midline=dict(x=q.x[0][order].tolist(), y=q.x[1][order].tolist(), v_y=v[1][order].tolist()))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--h", type=float, default=0.01)
    ap.add_argument("--layout", nargs="+", default=["hybrid"], choices=["hybrid", "regular", "scattered"])
    ap.add_argument("--Ra", type=float, default=1e6)
    ap.add_argument("--t-end", type=float, default=0.15)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--reports", type=int, default=30)
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    a = ap.parse_args(argv)
    res = []
    for lay in a.layout:
        r = run(h=a.h, layout=lay, Ra=a.Ra, t_end=a.t_end, tol=a.tol, reports=a.reports,
                progress=lambda s: print(s, file=sys.stderr, flush=True))
        print(json.dumps({k: r[k] for k in ("layout", "h", "N", "steps", "nu_final", "stepping_s",
                                            "krylov_iters_total")}), flush=True)
        res.append(r)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
