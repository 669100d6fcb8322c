"""The autotuner and the parameters it searches.

Every searched parameter changes only launch shapes, the node order and the
order of floating-point sums: stencils and weights must be bit-identical in
the caller's numbering, and fields after time steps equal to the FP64 field
tolerance.  The tuner must cover every parameter, and its cache must answer
a repeated call.
"""
import numpy as np
import pytest
import torch

from paper_2303_01760_amd import nodegen as ng

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-8


def _setup(s):
    dev = torch.device("cuda")
    x, kind, nrm = (torch.tensor(s.x, device=dev), torch.tensor(s.kind, device=dev),
                    torch.tensor(s.normal, device=dev))
    T0 = torch.tensor(np.where(s.kind == 1, s.tbc, 0.0), device=dev)
    v0 = torch.zeros((s.d, s.n), dtype=torch.float64, device=dev)
    return x, kind, nrm, v0, T0


def _run(s, knobs, steps=10):
    from paper_2303_01760_amd import hsm
    x, kind, nrm, v0, T0 = _setup(s)
    st = hsm.build_stencils(x, kind, nrm, s.h, 2, tile_log2=knobs.get("tile_log2", 0),
                            solve_groups=knobs.get("solve_groups", 0))
    ex = st.export()
    sim = hsm.Sim(st, v0, T0, Ra=1e5, Pr=0.71, dt=0.1 * s.h ** 2 / 2, T_ref=0.5, krylov_tol=1e-12,
                  krylov_maxiter=100000, block_nodes=knobs.get("block_nodes", 0),
                  gather_chunk=knobs.get("gather_chunk", 0), krylov_chunk=knobs.get("krylov_chunk", 0),
                  xcd_order=knobs.get("xcd_order", 0), reduce_mode=knobs.get("reduce_mode", 0),
                  wide_lanes=knobs.get("wide_lanes", 0))
    sim.step(steps)
    assert sim.stats()["status"] == 0
    out = [a.cpu().numpy() for a in sim.read()]
    sim.close()
    st.close()
    return ex, out


@pytest.mark.parametrize("knobs", [
    dict(tile_log2=2, solve_groups=1, block_nodes=64, gather_chunk=4, krylov_chunk=16),
    dict(tile_log2=4, solve_groups=2, block_nodes=128, gather_chunk=12, krylov_chunk=64, xcd_order=1,
         reduce_mode=2),
    dict(xcd_order=1, reduce_mode=2, wide_lanes=2),
    dict(wide_lanes=1, block_nodes=64),
    dict(wide_lanes=2, block_nodes=64, reduce_mode=1),
    dict(tile_log2=3, solve_groups=3, block_nodes=256, gather_chunk=6, krylov_chunk=32),
])
def test_searched_parameters_keep_results(knobs):
    s = ng.obstacles2d(h=0.01, n_obst=6, seed=11)
    ref_ex, ref = _run(s, {})
    ex, got = _run(s, knobs)
    for key in ("cls", "off", "idx", "w"):
        assert np.array_equal(ex[key], ref_ex[key]), key
    for a, b, name in zip(got, ref, ("v", "T", "p")):
        err = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        print(f"{knobs}: {name} rel diff {err:.2e}")
        assert err <= FIELD_TOL, (name, err)


def test_autotune_covers_every_parameter_and_caches(tmp_path):
    from paper_2303_01760_amd import autotune
    s = ng.obstacles2d(h=0.01, n_obst=6, seed=11)
    x, kind, nrm, v0, T0 = _setup(s)
    kw = dict(Ra=1e5, Pr=0.71, dt=0.1 * s.h ** 2 / 2, T_ref=0.5, tol=1e-10, v0=v0, T0=T0)
    path = str(tmp_path / "tune.json")
    r = autotune.tune(x, kind, nrm, s.h, 2, kw, path=path)
    assert not r["cached"]
    assert set(r["choice"]) == set(autotune.DEFAULTS)
    assert set(r["timings"]) == set(autotune.DEFAULTS), r["timings"].keys()
    for name, cands in r["timings"].items():
        assert len(cands) >= 2 and all(v > 0 for v in cands.values()), (name, cands)
    print(r["choice"], r["tuning_s"])
    again = autotune.tune(x, kind, nrm, s.h, 2, kw, path=path)
    assert again["cached"] and again["choice"] == r["choice"] and again["key"] == r["key"]
    # the tuned parameters give the default results
    ref_ex, ref = _run(s, {})
    ex, got = _run(s, r["choice"])
    assert np.array_equal(ex["w"], ref_ex["w"])
    for a, b in zip(got, ref):
        assert float(np.linalg.norm(a - b) / np.linalg.norm(b)) <= FIELD_TOL
