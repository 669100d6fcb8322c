"""De Vahl Davis cavity in the quarters layout (Section 4.1) on the GPU:
fields against the FP64 oracle after a short run, and the cold-wall Nusselt
number (Eq. (5)) the validation driver computes against the oracle's, from the
same fields."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2303_01760_amd import nodegen as ng

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-8


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("layout", ["hybrid", "scattered"])
def test_dvd_steps_and_nusselt_match_oracle(layout):
    from paper_2303_01760_amd import dvd, hsm
    q = ng.dvd2d(0.05, layout)
    dt = 0.1 * q.h ** 2 / 2
    prm = dict(Ra=1e5, Pr=0.71, dt=dt, T_ref=0.0)
    dev = torch.device("cuda")
    st = hsm.build_stencils(torch.tensor(q.x, device=dev), torch.tensor(q.kind, device=dev),
                            torch.tensor(q.normal, device=dev), q.h, 2)
    v0 = np.zeros((2, q.n))
    T0 = np.where(q.kind == ng.KIND_DIRICHLET, q.tbc, 0.0)
    sim = hsm.Sim(st, torch.tensor(v0, device=dev), torch.tensor(T0, device=dev), krylov_tol=1e-12, **prm)
    sim.step(40)
    assert sim.stats()["status"] == 0
    vg, Tg, pg = [a.cpu().numpy() for a in sim.read()]
    csr = O.to_csr(O.build(q.x, q.kind, q.normal, q.h, 2))
    vo, To, po = v0.copy(), T0.copy(), np.zeros(q.n + 1)
    O.Sim(csr, q.kind, solver=1).step(vo, To, po, 40, **prm)
    ev, eT, ep = _rel(vg, vo), _rel(Tg, To), _rel(pg, po[:q.n])
    cold = dvd.cold_wall_nodes(q)
    nu_g = dvd.nusselt(st, torch.tensor(Tg, device=dev), cold)
    nu_o = O.nusselt(csr, To, cold)
    print(f"dvd {layout}: N={q.n}, rel L2 err v {ev:.2e} T {eT:.2e} p {ep:.2e}; Nu gpu {nu_g:.12f} oracle {nu_o:.12f}")
    assert ev <= FIELD_TOL and eT <= FIELD_TOL and ep <= FIELD_TOL
    assert nu_g == pytest.approx(nu_o, rel=1e-9)
    # heat flows in through the hot wall and out through the cold one: Nu above conduction's 1 once convection starts
    assert nu_o > 1.0


def test_refined_obstacle_layout_build_and_steps_match_oracle():
    # Section 4.2's h-refined layout (spacing h_r/3 on the circles growing to
    # h_r over 4 h_r): classes, stencils and weights, then 20 steps, against
    # the oracle
    from paper_2303_01760_amd import hsm
    q = ng.refined2d(h_r=0.05, ratio=3, delta_h=4, n_obst=2, rmin=0.08, rmax=0.12, seed=91)
    dev = torch.device("cuda")
    st = hsm.build_stencils(torch.tensor(q.x, device=dev), torch.tensor(q.kind, device=dev),
                            torch.tensor(q.normal, device=dev), q.h, 2)
    ex = st.export()
    ora = O.to_csr(O.build(q.x, q.kind, q.normal, q.h, 2))
    assert np.array_equal(ex["cls"], ora["cls"])
    assert np.array_equal(ex["off"], ora["off"]) and np.array_equal(ex["idx"], ora["idx"])
    werr = np.abs(ex["w"][:3] - ora["w"]).max() / np.abs(ora["w"]).max()
    assert werr <= 1e-10
    h_s = q.h / 3
    prm = dict(Ra=1e5, Pr=0.71, dt=0.1 * h_s ** 2 / 2, T_ref=0.5)
    v0 = np.zeros((2, q.n))
    T0 = np.where(q.kind == ng.KIND_DIRICHLET, q.tbc, 0.0)
    sim = hsm.Sim(st, torch.tensor(v0, device=dev), torch.tensor(T0, device=dev), krylov_tol=1e-12, **prm)
    sim.step(20)
    assert sim.stats()["status"] == 0
    vg, Tg, pg = [a.cpu().numpy() for a in sim.read()]
    vo, To, po = v0.copy(), T0.copy(), np.zeros(q.n + 1)
    O.Sim(ora, q.kind, solver=1).step(vo, To, po, 20, **prm)
    ev, eT, ep = _rel(vg, vo), _rel(Tg, To), _rel(pg, po[:q.n])
    print(f"refined 2D: N={q.n}, weight rel err {werr:.1e}, fields v {ev:.2e} T {eT:.2e} p {ep:.2e}")
    assert ev <= FIELD_TOL and eT <= FIELD_TOL and ep <= FIELD_TOL


def test_checkpointed_run_continues_where_it_stopped(tmp_path):
    """A run stopped by its time budget and continued from its checkpoint
    reaches the same fields and Nusselt history as one uninterrupted run (the
    pressure border multiplier restarts from zero, so the two agree to the
    Krylov tolerance, not bit for bit)."""
    from paper_2303_01760_amd import dvd
    q = ng.dvd2d(0.05, "hybrid")
    dt = 0.1 * q.h ** 2 / 2
    kw = dict(Ra=1e5, T_ref=0.0, t_end=60 * dt, dt=dt, cold=dvd.cold_wall_nodes(q), tol=1e-12, reports=6)
    whole = dvd.run_case(q, **kw)
    ck = str(tmp_path / "ck.npz")
    part = dvd.run_case(q, **kw, checkpoint=ck, budget_s=0.0)     # stops after its first report
    assert not part["complete"] and part["steps"] == 10
    rest = dvd.run_case(q, **kw, checkpoint=ck)
    assert rest["complete"] and rest["steps"] == 60
    assert len(rest["nu_history"]) == len(whole["nu_history"])
    for (ta, na), (tb, nb) in zip(rest["nu_history"], whole["nu_history"]):
        assert abs(ta - tb) <= 1e-15 and abs(na - nb) <= 1e-8 * abs(nb)
    assert _rel(rest["v"], whole["v"]) <= FIELD_TOL and _rel(rest["T"], whole["T"]) <= FIELD_TOL
