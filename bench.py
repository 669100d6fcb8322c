#!/usr/bin/env python3
"""Benchmark of the hybrid scattered-regular hot path on one MI355X.

Workload: unit square minus 20 seeded circular obstacles (radii U(0.02, 0.08)),
lattice spacing h = 0.002, scattered band 0.05 around the obstacles, RBF-FD
PHS r^3 + m = 2 (n = 12) on scattered nodes, MON on the 5-node cross on
regular nodes; Ra = 1e5, Pr = 0.71, dt = 0.1 h^2 / 2 (the paper's rule).

One benchmark step is one pass of the whole hot path over the node set:
build the stencils and weights (neighbour search, classification, local
solves), apply d/dx, d/dy and the Laplacian to the three fields, then run
explicit Boussinesq time steps (predictor, BiCGSTAB pressure solve,
projection, heat transport, wall conditions).  The same steps are timed for
the hybrid layout and for the all-scattered layout on the same node set.

Prints one JSON line.  value = node-applies/s of the hybrid layout over the
timed region (every (operator, field, node) triple evaluated, Krylov
matrix-vector products included, divided by wall time).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stencil node-applies/s + weight solves/s, hybrid vs all-scattered, 1 GPU"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic_bicg_pv_obstacles2d_h0.002.json")
SIM_SRC = os.path.join(ROOT, "paper_2303_01760_amd", "csrc", "sim.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(sizes_buckets, N, D, kernel):
    """Algorithmic HBM bytes of one launch (FP64 values, int32 indices; every
    array element read or written once).  sizes_buckets: [(type, width, count)]."""
    nnz = sum(w * c for _, w, c in sizes_buckets)
    if kernel == "bicg_pv":    # idx + weights; gather s, t, p, v; read x, rh; write x, r, p, v
        return 12 * nnz + 80 * N
    if kernel == "bicg_st":    # idx + weights; gather r, v; read rh; write s, t
        return 12 * nnz + 40 * N
    raise ValueError(kernel)


def traffic_record():
    """Counter-measured bytes per launch of the dominant kernel, if taken on the current source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    sha = hashlib.sha256(open(SIM_SRC, "rb").read()).hexdigest()
    if rec.get("sim_source_sha256") != sha:
        return None
    return rec


def pmc_summary(fetch_csv, write_csv, out_path):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch)
    into HBM bytes per launch of k_bicg_pv, scaled by what the same counters
    read for the plain copy kernel (whose bytes are known exactly)."""
    import csv
    import statistics

    def per_kernel(path, counter):
        vals = {}
        for row in csv.DictReader(open(path)):
            if row.get("Counter_Name") != counter:
                continue
            name = row["Kernel_Name"]
            key = "pv" if "k_bicg_pv" in name else ("copy" if "k_stream_copy" in name else None)
            if key:
                vals.setdefault(key, []).append(float(row["Counter_Value"]) * 1024.0)
        return vals

    f, w = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy_bytes = float(1 << 31)            # each copy launch reads and writes 2 GiB
    f_scale = copy_bytes / statistics.median(f["copy"])
    w_scale = copy_bytes / statistics.median(w["copy"])
    # busy launches only (launches after convergence return at once)
    fb = sorted(f["pv"])[len(f["pv"]) // 2:]
    wb = sorted(w["pv"])[len(w["pv"]) // 2:]
    rec = dict(kernel="k_bicg_pv<2>", workload="2D unit square minus 20 circles, h=0.002, m=2, hybrid",
               fetch_bytes_per_launch=statistics.median(fb) * f_scale,
               write_bytes_per_launch=statistics.median(wb) * w_scale,
               copy_fetch_scale=f_scale, copy_write_scale=w_scale, launches=len(f["pv"]),
               sim_source_sha256=hashlib.sha256(open(SIM_SRC, "rb").read()).hexdigest())
    rec["hbm_bytes_per_launch"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    json.dump(rec, open(out_path, "w"), indent=1)
    print(json.dumps(rec))


def cpu_baseline(s, m, budget_s=12.0):
    """The FP64 oracle, single-threaded, on a seeded sample of the same node set."""
    import numpy as np
    from oracle import oracle as O
    rng = np.random.default_rng(2303017602)
    q = np.sort(rng.choice(s.n, 400, replace=False))
    t0 = time.perf_counter()
    st = O.build(s.x, s.kind, s.normal, s.h, m, queries=q)
    t_build = time.perf_counter() - t0
    width = st["width"].astype(np.int64)
    off = np.zeros(len(q) + 1, np.int64)
    np.cumsum(width, out=off[1:])
    mask = np.arange(st["idx"].shape[1])[None, :] < width[:, None]
    csr = dict(off=off, idx=st["idx"][mask].astype(np.int32))
    ws = [st["w"][:, r, :][mask] for r in range(3)]
    fields = [np.sin(3 * s.x[0]), np.cos(2 * s.x[1]), s.x[0] * s.x[1]]
    reps, applies, t_apply = 0, 0, 0.0
    while t_apply < budget_s and reps < 100000:
        t1 = time.perf_counter()
        for u in fields:
            for w in ws:
                O.apply(csr, w, u)
        t_apply += time.perf_counter() - t1
        reps += 1
        applies += 9 * len(q)
    return dict(value=applies / t_apply, unit="node-applies/s", cores=1, kind="oracle",
                sample=f"{len(q)} seeded nodes of the same node set: stencils and weights built by the oracle "
                       f"(brute-force neighbour search over all {s.n} nodes), then d/dx, d/dy, Laplacian applied "
                       f"to 3 fields {reps} times ({t_apply:.1f} s)",
                solves_per_s=len(q) / t_build, build_s=t_build)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--time-steps", type=int, default=5, help="explicit time steps per benchmark step")
    ap.add_argument("--m", type=int, default=2)
    ap.add_argument("--h", type=float, default=0.002)
    ap.add_argument("--tol", type=float, default=1e-10, help="relative residual of each pressure solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-all-scattered", action="store_true")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs into the traffic record and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], TRAFFIC_FILE)
        return 0
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (pass --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2303_01760_amd import hsm
    from paper_2303_01760_amd import nodegen as ng

    dev = torch.device("cuda:0")
    s = ng.obstacles2d(h=args.h)
    D = s.d
    x = torch.tensor(s.x, device=dev)
    kind = torch.tensor(s.kind, device=dev)
    nrm = torch.tensor(s.normal, device=dev)
    dt = 0.1 * s.h ** 2 / 2
    T0 = np.where(s.kind == 1, s.tbc, 0.0)
    v0 = torch.zeros((D, s.n), dtype=torch.float64, device=dev)
    T0d = torch.tensor(T0, device=dev)
    fields = [torch.tensor(np.sin(3 * s.x[0]), device=dev), torch.tensor(np.cos(2 * s.x[1]), device=dev), T0d]
    ops = hsm.OP_DX | hsm.OP_DY | hsm.OP_LAP
    log(f"node set: N={s.n}, h={s.h}, m={args.m}, dt={dt:.3e}")

    # achievable HBM bandwidth: plain copy of 2 GiB (also the byte-counter calibration kernel)
    src = torch.empty(1 << 28, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        hsm.stream_copy(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        hsm.stream_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    log(f"stream copy: {copy_gbs:.0f} GB/s")

    def one_step(mode, rec):
        t0 = time.perf_counter()
        st = hsm.build_stencils(x, kind, nrm, s.h, args.m, mode=mode)
        rec["build_s"] += time.perf_counter() - t0
        info = st.info()
        rec["build_dev_ms"] += info["build_ms"][0] + info["build_ms"][1] + info["build_ms"][2]
        rec["solve_dev_ms"] += info["build_ms"][2]
        out = torch.empty((3, s.n), dtype=torch.float64, device=dev)
        for f in fields:
            st.apply(st.to_internal(f), ops, hsm.F64, out=out)
        rec["applies"] += 3 * st.node_count(ops)
        sim = hsm.Sim(st, v0, T0d, Ra=1e5, Pr=0.71, dt=dt, T_ref=0.5, krylov_tol=args.tol, krylov_maxiter=200000,
                      profile=1)
        sim.step(args.time_steps)
        stats = sim.stats()
        assert stats["status"] == 0, stats
        rec["applies"] += stats["node_applies"]
        rec["krylov_iters"] += stats["krylov_iters_total"]
        rec["solves"] += s.n
        rec["info"] = info
        rec["ktimes"] = sim.kernel_times()
        rec["sizes"] = sim.sizes()
        return st

    results = {}
    modes = [("hybrid", hsm.MODE_HYBRID)] + ([] if args.skip_all_scattered else [("all_scattered", hsm.MODE_ALL_SCATTERED)])
    for name, mode in modes:
        rec = dict(build_s=0.0, build_dev_ms=0.0, solve_dev_ms=0.0, applies=0, krylov_iters=0, solves=0)
        for _ in range(args.warmup):
            one_step(mode, dict(rec))
        torch.cuda.synchronize()
        rec = dict(build_s=0.0, build_dev_ms=0.0, solve_dev_ms=0.0, applies=0, krylov_iters=0, solves=0)
        t0 = time.perf_counter()
        for k in range(args.steps):
            one_step(mode, rec)
            log(f"{name}: step {k + 1}/{args.steps} done")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rec["elapsed_s"] = el
        results[name] = rec
        log(f"{name}: {el / args.steps * 1e3:.1f} ms/step, {rec['applies'] / el:.3e} node-applies/s, "
            f"krylov iters/step {rec['krylov_iters'] / args.steps:.0f}")

    hy = results["hybrid"]
    info = hy["info"]
    buckets = info["buckets"]
    kt = hy["ktimes"]
    dom = max(("bicg_pv", "bicg_st"), key=lambda k: kt[k][0])
    bytes_launch = kernel_bytes(buckets, s.n, D, dom)
    mean_ms = kt[dom][0]
    achieved = bytes_launch / (mean_ms * 1e-3) / 1e9
    tr = traffic_record() if dom == "bicg_pv" else None
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=(tr["hbm_bytes_per_launch"] if tr else None), kernel="k_bicg_pv<2>" if dom == "bicg_pv"
                    else "k_bicg_st<2>", bytes_per_launch=bytes_launch, mean_launch_ms=mean_ms,
                    launches_timed=kt[dom][1], copy_kernel_gbs=copy_gbs)
    el = hy["elapsed_s"]
    out = dict(metric=METRIC, value=hy["applies"] / el, unit="node-applies/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=el / args.steps * 1e3, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload=f"2D unit square minus 20 seeded circles, h={s.h}, band 0.05, m={args.m} "
                                    f"(n={2 * (args.m + 1) * (args.m + 2) // 2}), hybrid; per step: stencil build + "
                                    f"3-field apply + {args.time_steps} Boussinesq steps (Ra=1e5, Pr=0.71, "
                                    f"dt=0.1h^2/2, pressure rel. residual {args.tol})",
                           nodes=s.n, n_regular=info["n_regular"], n_scattered=info["n_scattered"],
                           time_steps_per_step=args.time_steps, krylov_tol=args.tol),
               solves_per_s=hy["solves"] / hy["build_s"], solves_per_s_device=hy["solves"] / (hy["solve_dev_ms"] * 1e-3),
               krylov_iters_per_time_step=hy["krylov_iters"] / (args.steps * args.time_steps),
               kernel_mean_ms={k: v[0] for k, v in kt.items()},
               roofline=roofline)
    if "all_scattered" in results:
        a = results["all_scattered"]
        out["all_scattered"] = dict(value=a["applies"] / a["elapsed_s"], ms_per_step=a["elapsed_s"] / args.steps * 1e3,
                                    krylov_iters_per_time_step=a["krylov_iters"] / (args.steps * args.time_steps),
                                    solves_per_s=a["solves"] / a["build_s"],
                                    solves_per_s_device=a["solves"] / (a["solve_dev_ms"] * 1e-3),
                                    kernel_mean_ms={k: v[0] for k, v in a["ktimes"].items()})
        out["hybrid_speedup_per_step"] = a["elapsed_s"] / el
        # per-iteration cost ratio of the pressure operator (same node set, same kernels)
        out["hybrid_speedup_per_krylov_iteration"] = (a["ktimes"]["bicg_pv"][0] + a["ktimes"]["bicg_st"][0]) / \
            (kt["bicg_pv"][0] + kt["bicg_st"][0])
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(s, args.m)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
