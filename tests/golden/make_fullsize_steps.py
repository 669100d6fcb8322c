"""Write fullsize_steps_obstacles2d_h0.002.npz: the FP64 oracle's fields after
three explicit Boussinesq steps (Section 3, Eqs. (2)-(4)) on the full 2D
20-circle node set at h = 0.002 (167 231 nodes), m = 2, in the hybrid and the
all-scattered layouts, at a seeded sample of nodes, with full-field norms.

Only the oracle (oracle/) and the node generator run here; nothing comes from
the GPU library.  The oracle's brute-force stencil build is split over worker
processes by node (each runs the oracle unchanged on its share of the
queries); the time steps run in one process per layout.  About 7 minutes on 8
cores.  The GPU test test_full_size_steps_match_oracle compares against it.

Usage: python tests/golden/make_fullsize_steps.py [--procs N]
"""
import argparse
import hashlib
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2303_01760_amd import nodegen as ng  # noqa: E402

OUT = os.path.join(HERE, "fullsize_steps_obstacles2d_h0.002.npz")
PARAMS = dict(Ra=1e5, Pr=0.71, T_ref=0.5, tol=1e-12, steps=3, m=2, h=0.002, sample=4096, seed=2303017612)


def nodeset():
    return ng.obstacles2d(h=PARAMS["h"])


def nodeset_sha(s):
    h = hashlib.sha256()
    for a in (s.x, s.kind, s.normal, s.tbc):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _build_part(args):
    mode, q = args
    s = nodeset()
    return O.build(s.x, s.kind, s.normal, s.h, PARAMS["m"], mode=mode, queries=q)


def _steps(mode_parts):
    mode, parts = mode_parts
    s = nodeset()
    st = {k: np.concatenate([p[k] for p in parts]) for k in ("cls", "width", "idx", "w", "wn")}
    st["d"] = s.d
    csr = O.to_csr(st)
    sim = O.Sim(csr, s.kind)
    v = np.zeros((s.d, s.n))
    T = np.where(s.kind == ng.KIND_DIRICHLET, s.tbc, 0.0)
    p = np.zeros(s.n + 1)
    dt = 0.1 * s.h ** 2 / 2
    its = sim.step(v, T, p, PARAMS["steps"], Ra=PARAMS["Ra"], Pr=PARAMS["Pr"], dt=dt, T_ref=PARAMS["T_ref"],
                   tol=PARAMS["tol"], maxiter=200000)
    return mode, v, T, p[:s.n], its


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 4)
    a = ap.parse_args()
    t0 = time.time()
    s = nodeset()
    chunks = np.array_split(np.arange(s.n), 8 * a.procs)
    modes = (O.HYBRID, O.ALL_SCATTERED)
    with Pool(a.procs) as pool:
        parts = pool.map(_build_part, [(mode, q) for mode in modes for q in chunks])
        print(f"stencils built ({time.time() - t0:.0f} s)", flush=True)
        per = len(chunks)
        res = pool.map(_steps, [(mode, parts[k * per:(k + 1) * per]) for k, mode in enumerate(modes)])
    print(f"steps done ({time.time() - t0:.0f} s)", flush=True)
    rng = np.random.default_rng(PARAMS["seed"])
    walls = np.where(s.kind != 0)[0]
    inner = np.where(s.kind == 0)[0]
    sample = np.sort(np.concatenate([rng.choice(inner, PARAMS["sample"] * 3 // 4, replace=False),
                                     rng.choice(walls, PARAMS["sample"] // 4, replace=False)]))
    out = dict(sample=sample.astype(np.int64), nodeset_sha256=np.array(nodeset_sha(s)), n=np.array(s.n),
               params=np.array(repr(PARAMS)))
    for mode, v, T, p, its in res:
        tag = "hybrid" if mode == O.HYBRID else "all_scattered"
        out[f"{tag}_v"] = v[:, sample]
        out[f"{tag}_T"] = T[sample]
        out[f"{tag}_p"] = p[sample]
        out[f"{tag}_norms"] = np.array([np.linalg.norm(v[0]), np.linalg.norm(v[1]), np.linalg.norm(T),
                                        np.linalg.norm(p)])
        out[f"{tag}_iters"] = its.astype(np.int64)
        print(f"{tag}: iterations {its.tolist()}, |u| {np.linalg.norm(v[0]):.6e}", flush=True)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} ({os.path.getsize(OUT)} bytes, {time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
