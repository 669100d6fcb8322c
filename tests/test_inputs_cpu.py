"""Checks of the seeded input generators (CPU only).

The 512-domain batch must hold node sets the explicit scheme can step: its
smallest domains (the coarsest, whose circles span the fewest node spacings)
are stepped by the oracle from rest and must stay physical.
"""
import numpy as np

from oracle import oracle as O
from paper_2303_01760_amd import nodegen as ng


def test_smallest_batch_domains_step_stably():
    b = ng.batch2d()
    counts = np.diff(b.off)
    dt = 0.1 * float(np.min(b.h)) ** 2 / 2          # the batch's common time step
    for k in np.argsort(counts)[:3]:
        a, e = int(b.off[k]), int(b.off[k + 1])
        x, kind, nrm = b.x[:, a:e].copy(), b.kind[a:e].copy(), b.normal[:, a:e].copy()
        csr = O.to_csr(O.build(x, kind, nrm, float(b.h[k]), int(b.m[k])))
        v = np.zeros((2, e - a))
        T = np.where(kind == 1, b.tbc[a:e], 0.0)
        p = np.zeros(e - a + 1)
        sim = O.Sim(csr, kind, solver=1)
        sim.step(v, T, p, 5, 1e5, 0.71, dt, 0.5, tol=1e-10, maxiter=200000)
        # buoyancy alone from rest: |v| ~ Ra Pr |T - T_ref| t = 0.14 after five steps
        assert np.isfinite(v).all() and np.abs(v).max() < 1.0, (int(k), float(np.abs(v).max()))
        assert np.abs(T).max() <= 1.0 + 1e-9


def test_fill_keeps_half_a_spacing_from_the_box():
    # interior fill nodes stay at least half the local spacing (>= h_s / 2)
    # from every box face, also along the 3D box edges where no wall nodes are
    from paper_2303_01760_amd.irregular import node_set
    for dim, ratio in ((3, 2.0), (2, 3.0)):
        q = node_set(dim, "scattered", 4.0)
        h_s = q.h / ratio
        fill = q.kind == 0
        gap = np.minimum(q.x[:, fill], 1.0 - q.x[:, fill]).min()
        assert gap >= 0.5 * h_s * (1 - 1e-12), (dim, float(gap), h_s)


def test_full_size_step_fixture_matches_the_generator():
    """The stored oracle fields of the full-size step test were computed on the
    node set the generator makes now (else regenerate them with
    tests/golden/make_fullsize_steps.py)."""
    import hashlib
    import os
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", "fullsize_steps_obstacles2d_h0.002.npz"))
    s = ng.obstacles2d(h=0.002)
    sha = hashlib.sha256()
    for a in (s.x, s.kind, s.normal, s.tbc):
        sha.update(np.ascontiguousarray(a).tobytes())
    assert sha.hexdigest() == str(z["nodeset_sha256"])
    assert int(z["n"]) == s.n == 167231
    S = z["sample"]
    assert len(S) == len(np.unique(S)) == 4096 and S.min() >= 0 and S.max() < s.n
    for tag in ("hybrid", "all_scattered"):
        assert z[f"{tag}_v"].shape == (2, len(S)) and np.all(np.isfinite(z[f"{tag}_v"]))
        # walls are no-slip in the stored fields
        assert np.all(z[f"{tag}_v"][:, s.kind[S] != 0] == 0.0)
