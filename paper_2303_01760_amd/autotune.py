"""Autotuner for the layout of the internal node order.

The library stores nodes width bucket by width bucket and, inside a bucket,
in the order of the neighbour-search cells, numbered tile by tile (tiles of
2^L cells per axis, row-major).  The tile edge decides how compact a block of
256 consecutive nodes is in space, and so how many of the values its stencils
gather are already in the L2 cache of the XCD that runs it.  tune_tile builds
the stencils once per candidate L and times the fused apply of d/dx, d/dy
(, d/dz) and the Laplacian to one field (mean of `reps` launches replayed
from a graph between events, after warm-up; the median of five replays).  It leaves the default only for
a candidate faster by more than `margin`: differences within the noise of
the timing would otherwise pick at random, and the pressure iteration, which
gathers other vectors through the same order, need not follow the apply's
small differences (measured: a 3D pick worth 0.4 % on the apply cost 8 % on
the iteration).
"""
from __future__ import annotations

import torch

from . import hsm

DEFAULT_CANDIDATES = {2: (2, 3, 4), 3: (1, 2, 3)}
DEFAULT_TILE = {2: 3, 3: 2}


def _time_apply(st: hsm.Stencils, d: int, reps: int) -> float:
    """Mean time of one fused apply: reps launches captured in a graph and replayed between events, so the
    host's per-launch cost does not leave the device idle between short launches."""
    ops = hsm.OP_DX | hsm.OP_DY | hsm.OP_LAP | (hsm.OP_DZ if d == 3 else 0)
    nops = bin(ops).count("1")
    dev = torch.device("cuda")
    gen = torch.Generator(device="cpu").manual_seed(2303017600)
    u = torch.rand(st.n, generator=gen, dtype=torch.float64).to(dev)
    out = torch.empty((nops, st.n), dtype=torch.float64, device=dev)
    for _ in range(3):              # also uploads the launch tables before the capture
        st.apply(u, ops, hsm.F64, out=out)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(reps):
                st.apply(u, ops, hsm.F64, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    graph.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(5):              # the median of five replays: one disturbed replay does not decide
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / reps)
    del graph
    return sorted(times)[len(times) // 2]


def tune_tile(x: torch.Tensor, kind: torch.Tensor, normal: torch.Tensor, h, m, mode=hsm.MODE_HYBRID,
              domain_offsets=None, n=None, candidates=None, reps: int = 20, margin: float = 0.05):
    """Return (chosen tile_log2, {tile_log2: mean apply ms}) for this node set."""
    d = int(x.shape[0])
    cands = tuple(candidates) if candidates is not None else DEFAULT_CANDIDATES[d]
    times = {}
    for L in cands:
        st = hsm.build_stencils(x, kind, normal, h, m, mode=mode, domain_offsets=domain_offsets, n=n, tile_log2=L)
        times[L] = _time_apply(st, d, reps)
        st.close()
    best = min(times, key=times.get)
    dflt = DEFAULT_TILE[d]
    if dflt in times and times[best] > (1.0 - margin) * times[dflt]:
        best = dflt
    return best, times
