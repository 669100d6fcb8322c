"""FP32 field form against the FP64 form over many time steps.

The same node set and initial state are stepped twice on the GPU, once with
FP64 fields and once in the FP32 form (FP32 v and T, compensated Dot2
applies, FP64 pressure), in lockstep; every `report` steps the fields of the
two runs are compared: maximum relative error (max |a - b| / max |b|) and
relative L2 error of each velocity component, of T, and of p after removing
its mean.  The default is the 2D obstacle domain at h = 0.001 with m = 4
(n = 30) at Ra = 1e6 for 500 steps.

Usage:
    python -m paper_2303_01760_amd.precision --h 0.001 --m 4 --Ra 1e6 --steps 500 --out <file>
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import hsm
from . import nodegen as ng


def _err(a: np.ndarray, b: np.ndarray) -> dict:
    return dict(max_rel=float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)),
                rel_l2=float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)))


def compare(h: float = 0.001, m: int = 4, Ra: float = 1e6, steps: int = 500, report: int = 50,
            tol: float = 1e-10, budget_s: float = 1e30, progress=None) -> dict:
    q = ng.obstacles2d(h=h)
    dev = torch.device("cuda")
    st = hsm.build_stencils(torch.tensor(q.x, device=dev), torch.tensor(q.kind, device=dev),
                            torch.tensor(q.normal, device=dev), q.h, m)
    dt = 0.1 * h * h / 2
    v0 = torch.zeros((2, q.n), dtype=torch.float64, device=dev)
    T0 = torch.tensor(np.where(q.kind == ng.KIND_DIRICHLET, q.tbc, 0.0), device=dev)
    prm = dict(Ra=Ra, Pr=0.71, dt=dt, T_ref=0.5, krylov_tol=tol, krylov_maxiter=200000)
    sims = {"f64": hsm.Sim(st, v0, T0, field_dtype=hsm.F64, **prm),
            "f32_comp": hsm.Sim(st, v0, T0, field_dtype=hsm.F32_COMP, **prm)}
    hist, done, t0 = [], 0, time.perf_counter()
    status = "ok"
    while done < steps:
        k = min(report, steps - done)
        try:
            for s in sims.values():
                s.step(k)
        except hsm.HsmError as e:
            status = f"stepping failed: {e}"
            break
        torch.cuda.synchronize()
        done += k
        got = {name: [a.cpu().numpy() for a in s.read()] for name, s in sims.items()}
        (v64, T64, p64), (v32, T32, p32) = got["f64"], got["f32_comp"]
        if not (np.all(np.isfinite(v32)) and np.all(np.isfinite(T32)) and np.all(np.isfinite(p32))):
            status = "non-finite FP32-form fields"
        rec = dict(step=done, t=done * dt, u=_err(v32[0], v64[0]), v=_err(v32[1], v64[1]), T=_err(T32, T64),
                   p=_err(p32 - p32.mean(), p64 - p64.mean()),
                   krylov_iters=dict((n, s.stats()["krylov_iters_total"]) for n, s in sims.items()))
        hist.append(rec)
        if progress:
            progress(f"step {done}/{steps}: rel L2 u {rec['u']['rel_l2']:.2e} v {rec['v']['rel_l2']:.2e} "
                     f"T {rec['T']['rel_l2']:.2e} p {rec['p']['rel_l2']:.2e} ({time.perf_counter() - t0:.0f} s)")
        if status != "ok":
            break
        if time.perf_counter() - t0 > budget_s and done < steps:
            status = f"stopped at step {done} (time budget)"
            break
    for s in sims.values():
        s.close()
    st.close()
    return dict(case=f"2D unit square minus 20 circles, h={h}, m={m}, Ra={Ra:g}, Pr=0.71, dt=0.1h^2/2, "
                     f"pressure rel. residual {tol}", N=q.n, steps=done, status=status, history=hist,
                final=hist[-1] if hist else None)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--h", type=float, default=0.001)
    ap.add_argument("--m", type=int, default=4)
    ap.add_argument("--Ra", type=float, default=1e6)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--report", type=int, default=50)
    ap.add_argument("--tol", type=float, default=1e-10, help="relative residual of the pressure solves")
    ap.add_argument("--budget-s", type=float, default=1e30, help="stop (and say so) after this much stepping time")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    r = compare(h=a.h, m=a.m, Ra=a.Ra, steps=a.steps, report=a.report, tol=a.tol, budget_s=a.budget_s,
                progress=lambda s: print(s, file=sys.stderr, flush=True))
    print(json.dumps(dict(N=r["N"], steps=r["steps"], status=r["status"], final=r["final"])), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(r, f, indent=1)


if __name__ == "__main__":
    main()
