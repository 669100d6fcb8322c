"""Pins of the FP64 CPU oracle against facts fixed by the paper or by mathematics.

Each test checks the oracle against something other than itself: values the
paper prints, closed forms, exactness properties, a library routine on a case
the method reduces to, or brute force.  CPU only.
"""
import json
import os
from math import comb

import numpy as np
import pytest

from oracle import oracle as O
from paper_2303_01760_amd import nodegen as ng

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# ------------------------------------------------------------- sizes / dt --
def test_stencil_sizes_match_paper():
    g = GOLD["stencil_sizes"]
    assert O.stencil_size(2, 2) == g["rbffd_2d_m2"]
    assert O.stencil_size(2, 4) == 30 and O.stencil_size(3, 2) == 20
    assert 2 * 2 + 1 == g["mon_2d"] and 2 * 3 + 1 == g["mon_3d"]


def test_dt_rule_reproduces_printed_value():
    g = GOLD["dt_rule"]
    h_s = g["h_r"] * g["h_s_over_h_r"]
    assert 0.1 * h_s ** 2 / 2 == pytest.approx(g["dt_printed"], rel=1e-15)


def test_monomial_order_and_count():
    for d, m in ((2, 2), (2, 4), (3, 2), (3, 3)):
        al = O.monomials(d, m)
        assert len(al) == comb(m + d, d)
        deg = al.sum(1)
        assert np.all(np.diff(deg) >= 0)               # graded
        assert len({tuple(a) for a in al}) == len(al)  # distinct
    assert O.monomials(2, 2).tolist() == [[0, 0], [1, 0], [0, 1], [2, 0], [1, 1], [0, 2]]


# ------------------------------------------------------------------- kNN ----
def _brute_knn(x, i, k, cand):
    dx = x[:, cand] - x[:, [i]]
    d2 = dx[0] * dx[0]
    for a in range(1, x.shape[0]):
        d2 = d2 + dx[a] * dx[a]
    order = np.lexsort((cand, d2))
    return cand[order[:k]]


@pytest.mark.parametrize("d,n,k", [(2, 300, 12), (2, 250, 30), (3, 400, 20)])
def test_knn_matches_sort_based_brute_force(d, n, k):
    s = ng.random_cloud(n, d, seed=7 + d)
    got = O.knn(s.x, k)
    allj = np.arange(n)
    for i in range(n):
        np.testing.assert_array_equal(got[i], _brute_knn(s.x, i, k, allj))
    assert np.all(got[:, 0] == np.arange(n))


def test_knn_multi_domain_and_boundary_rule():
    rng = np.random.default_rng(3)
    x = rng.random((2, 200))
    kind = (rng.random(200) < 0.3).astype(np.uint8)
    off = np.array([0, 90, 200])
    got = O.knn(x, 12, dom_off=off, kind=kind)
    for i in range(200):
        lo, hi = (0, 90) if i < 90 else (90, 200)
        cand = np.arange(lo, hi)
        if kind[i]:
            cand = cand[(kind[cand] == 0) | (cand == i)]
        np.testing.assert_array_equal(got[i], _brute_knn(x, i, 12, cand))


def test_knn_lattice_ties_by_index():
    # 12 nearest of a lattice node: itself, 4 at h, 4 at sqrt(2)h, then 3 of the 4 at 2h (lowest indices).
    h = 0.125
    ii, jj = np.meshgrid(np.arange(9), np.arange(9), indexing="xy")
    x = np.stack([ii.ravel() * h, jj.ravel() * h]).astype(np.float64)
    c = 4 * 9 + 4
    got = O.knn(x, 12, queries=[c])[0]
    def at(i, j):
        return j * 9 + i
    expect = [c, at(4, 3), at(3, 4), at(5, 4), at(4, 5),
              at(3, 3), at(5, 3), at(3, 5), at(5, 5),
              at(4, 2), at(2, 4), at(6, 4)]
    assert got.tolist() == expect


def test_knn_duplicate_node_is_an_error():
    s = ng.random_cloud(50, 2, seed=1)
    s.x[:, 20] = s.x[:, 33]
    with pytest.raises(O.OracleError) as e:
        O.knn(s.x, 12)
    assert e.value.code == O.E_DUPLICATE and e.value.node == 20


# -------------------------------------------------------------- classify ----
def test_classifier_on_lattice_with_hole():
    # 9x9 lattice; the outer ring lacks a complete cross, and so do the four
    # neighbours of the removed node (4,4): regular = 7*7 - 1 (hole) - 4.
    h = 0.1
    pts = [(i * h, j * h) for j in range(9) for i in range(9) if (i, j) != (4, 4)]
    x = np.array(pts).T.copy()
    kind = np.zeros(x.shape[1], np.uint8)
    cls, cross = O.classify(x, kind, h)
    assert int((cls == 0).sum()) == 49 - 1 - 4
    # a regular node's cross is [c, -x, +x, -y, +y]
    k = int(np.where(cls == 0)[0][0])
    xc = x[:, cross[k]] - x[:, [k]]
    np.testing.assert_allclose(xc.T, [[0, 0], [-h, 0], [h, 0], [0, -h], [0, h]], atol=1e-12)
    # a boundary node is never regular
    kind[k] = 2
    cls2, _ = O.classify(x, kind, h)
    assert cls2[k] == 1


def test_cavity_regular_count():
    # lattice kept for indices 5..45 along both axes (band 0.1 at h = 0.02): the
    # outermost kept ring lacks a complete cross, leaving 39^2 regular nodes
    s = ng.cavity2d()
    cls, _ = O.classify(s.x, s.kind, s.h)
    assert int((cls == 0).sum()) == 39 ** 2


# -------------------------------------------------------------- dense LU ----
def test_dense_lu_against_lapack():
    rng = np.random.default_rng(11)
    for S in (5, 18, 45):
        a = rng.standard_normal((S, S))
        b = rng.standard_normal((S, 3))
        np.testing.assert_allclose(O.dense_lu_solve(a, b), np.linalg.solve(a, b), rtol=1e-9, atol=1e-11)


def test_dense_lu_singular():
    a = np.ones((4, 4))
    with pytest.raises(O.OracleError) as e:
        O.dense_lu_solve(a, np.ones(4))
    assert e.value.code == O.E_SINGULAR


# ------------------------------------------------------------------- MON ----
def test_mon_central_difference_closed_form():
    h = 0.013
    xc = np.array([0.3, 0.7])
    xs = np.array([xc, xc - [h, 0], xc + [h, 0], xc - [0, h], xc + [0, h]])
    w = O.mon(xs)
    np.testing.assert_allclose(w[0], [0, -1 / (2 * h), 1 / (2 * h), 0, 0], atol=1e-8 / h)
    np.testing.assert_allclose(w[1], [0, 0, 0, -1 / (2 * h), 1 / (2 * h)], atol=1e-8 / h)
    np.testing.assert_allclose(w[2], [-4 / h ** 2] + [1 / h ** 2] * 4, rtol=1e-9)


def test_mon_3d_closed_form():
    h = 0.02
    xc = np.array([0.5, 0.25, 0.75])
    xs = [xc]
    for a in range(3):
        for s in (-1, 1):
            p = xc.copy(); p[a] += s * h; xs.append(p)
    w = O.mon(np.array(xs))
    for a in range(3):
        ref = np.zeros(7); ref[1 + 2 * a] = -1 / (2 * h); ref[2 + 2 * a] = 1 / (2 * h)
        np.testing.assert_allclose(w[a], ref, atol=1e-8 / h)
    np.testing.assert_allclose(w[3], [-6 / h ** 2] + [1 / h ** 2] * 6, rtol=1e-9)


# ---------------------------------------------------------------- RBF-FD ----
def _random_stencil(d, n, seed, scale=0.01):
    rng = np.random.default_rng(seed)
    xc = rng.random(d)
    pts = xc + scale * (rng.random((n - 1, d)) - 0.5) * 4
    return np.vstack([xc, pts])


def _mono(al, y):
    p = np.ones(y.shape[0])
    for a, e in enumerate(al):
        p = p * y[:, a] ** e
    return p


@pytest.mark.parametrize("d,m", [(2, 2), (2, 4), (3, 2)])
def test_rbffd_reproduces_polynomials(d, m):
    n = O.stencil_size(d, m)
    for seed in range(5):
        xs = _random_stencil(d, n, seed)
        w = O.rbffd(xs, m)
        y = xs - xs[0]
        for al in O.monomials(d, m):
            u = _mono(al, y)
            scale = np.abs(w).sum(1) * np.abs(u).max() + 1e-300
            # exact derivatives of y^alpha at y = 0
            for a in range(d):
                ref = 1.0 if (al.sum() == 1 and al[a] == 1) else 0.0
                assert abs(w[a] @ u - ref) <= 1e-11 * max(scale[a], 1.0)
            ref = 2.0 if (al.sum() == 2 and al.max() == 2) else 0.0
            assert abs(w[d] @ u - ref) <= 1e-11 * max(scale[d], 1.0)


@pytest.mark.parametrize("d,m", [(2, 2), (2, 4), (3, 2)])
def test_rbffd_exact_on_the_phs_interpolation_space(d, m):
    # u(x) = sum_j lam_j |x - x_j|^3 with P^T lam = 0 lies in the RBF-FD
    # interpolation space, so the weights reproduce its derivatives at the
    # centre exactly.  Analytic derivatives of |x - x_j|^3:
    #   d/dx_a = 3 |x - x_j| (x - x_j)_a,   Lap = 3 (d + 1) |x - x_j|.
    n = O.stencil_size(d, m)
    xs = _random_stencil(d, n, 42)
    w = O.rbffd(xs, m)
    y = xs - xs[0]
    P = np.stack([_mono(a, y) for a in O.monomials(d, m)], axis=1)
    null = np.linalg.svd(P.T)[2][P.shape[1]:].T          # basis of null(P^T), via LAPACK
    rng = np.random.default_rng(1)
    for _ in range(3):
        lam = null @ rng.standard_normal(null.shape[1])
        R = np.linalg.norm(xs[:, None, :] - xs[None, :, :], axis=2)
        u = (R ** 3) @ lam
        dc = xs[0] - xs                                   # [n, d]
        rc = np.linalg.norm(dc, axis=1)
        for a in range(d):
            ref = (3 * rc * dc[:, a]) @ lam
            assert abs(w[a] @ u - ref) <= 1e-9 * (np.abs(w[a]).sum() * np.abs(u).max() + abs(ref))
        ref = (3 * (d + 1) * rc) @ lam
        assert abs(w[d] @ u - ref) <= 1e-9 * (np.abs(w[d]).sum() * np.abs(u).max() + abs(ref))
    # a lone |x - x_k|^3 is not in the space (P^T e_k != 0): not reproduced
    u = np.linalg.norm(xs - xs[1], axis=1) ** 3
    assert abs(w[d] @ u - 3 * (d + 1) * np.linalg.norm(xs[0] - xs[1])) > 1e-6 * np.abs(w[d]).sum() * u.max()


def test_rbffd_square_polynomial_case_reduces_to_vandermonde():
    # With exactly Q nodes, P^T w = l_p alone fixes the weights (P square).
    d, m = 2, 2
    Q = comb(m + d, d)
    xs = _random_stencil(d, Q, 5)
    w = O.rbffd(xs, m)
    y = xs - xs[0]
    al = O.monomials(d, m)
    P = np.stack([_mono(a, y) for a in al], axis=1)  # [n, Q]
    l = np.zeros((Q, d + 1))
    for q, a in enumerate(al):
        for ax in range(d):
            if a.sum() == 1 and a[ax] == 1:
                l[q, ax] = 1.0
            if a.sum() == 2 and a[ax] == 2:
                l[q, d] = 2.0
    ref = np.linalg.solve(P.T, l).T
    np.testing.assert_allclose(w, ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


def test_rbffd_scale_and_translation_invariance():
    xs = _random_stencil(2, 12, 9)
    w = O.rbffd(xs, 2)
    s, t = 3.5, np.array([10.0, -4.0])
    w2 = O.rbffd(xs * s + t, 2)
    np.testing.assert_allclose(w2[:2] * s, w[:2], rtol=1e-8, atol=1e-9 * np.abs(w[:2]).max())
    np.testing.assert_allclose(w2[2] * s * s, w[2], rtol=1e-8, atol=1e-9 * np.abs(w[2]).max())


def test_rbffd_symmetric_stencil_gives_antisymmetric_gradient():
    h = 0.01
    c = np.array([0.5, 0.5])
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1), (-1, -1), (1, 1), (-1, 1), (1, -1), (-2, 0), (2, 0), (0, 2)]
    xs = c + h * np.array(offs, float)
    w = O.rbffd(xs, 2)
    # mirror x -> -x swaps nodes 1<->2, 5<->8(?): check the pair (-1,0)/(1,0)
    assert w[0][1] == pytest.approx(-w[0][2], rel=1e-9)
    assert w[0][9] == pytest.approx(-w[0][10], rel=1e-9)
    assert abs(w[0].sum()) < 1e-9 * np.abs(w[0]).sum()
    assert abs(w[2].sum()) < 1e-9 * np.abs(w[2]).sum()


def test_rbffd_collinear_is_singular():
    xs = np.stack([np.linspace(0, 1, 12), np.zeros(12)], 1)
    with pytest.raises(O.OracleError) as e:
        O.rbffd(xs, 2)
    assert e.value.code == O.E_SINGULAR


# --------------------------------------------------------- build / apply ----
def test_build_hybrid_cavity_reproduces_quadratics():
    s = ng.cavity2d()
    st = O.build(s.x, s.kind, s.normal, s.h, 2)
    csr = O.to_csr(st)
    x, y = s.x
    for u, ref in ((x * x, (2 * x, 0 * x, 2 + 0 * x)), (x * y, (y, x, 0 * x)), (y * y - 3 * x, (-3 + 0 * x, 2 * y, 2 + 0 * x))):
        for r in range(3):
            err = np.abs(O.apply(csr, csr["w"][r], u) - ref[r]).max()
            assert err < 1e-9 * max(1.0, np.abs(ref[r]).max()) * (1 if r < 2 else 1 / s.h)
    # regular nodes use the 5-node cross, everything else 12 nodes
    assert set(np.unique(st["width"][st["cls"] == 0])) == {5}
    assert set(np.unique(st["width"][st["cls"] == 1])) == {12}
    # boundary stencils couple to interior nodes only
    bnd = np.where(s.kind != 0)[0]
    assert np.all(s.kind[st["idx"][bnd, 1:12]] == 0)


def test_normal_derivative_weights():
    s = ng.cavity2d()
    st = O.build(s.x, s.kind, s.normal, s.h, 2)
    csr = O.to_csr(st)
    x, y = s.x
    u = 2 * x - 5 * y + x * y
    dn = s.normal[0] * (2 + y) + s.normal[1] * (-5 + x)
    got = O.apply(csr, csr["wn"], u)
    bnd = s.kind != 0
    np.testing.assert_allclose(got[bnd], dn[bnd], atol=1e-8)
    assert np.all(got[~bnd] == 0)


def test_manufactured_poisson_converges():
    # -Lap u = f, u = sin(pi x) sin(pi y), Dirichlet data on the box walls; the
    # global error of the hybrid discretisation falls at about second order.
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    errs, hs = [], []
    for h in (0.05, 0.025, 0.0125):
        s = ng.cavity2d(h=h, wall_band=0.1)
        st = O.build(s.x, s.kind, s.normal, s.h, 2)
        csr = O.to_csr(st)
        N = s.n
        x, y = s.x
        u = np.sin(np.pi * x) * np.sin(np.pi * y)
        f = 2 * np.pi ** 2 * u
        rows = np.repeat(np.arange(N), np.diff(csr["off"]))
        A = sp.csr_matrix((csr["w"][2], (rows, csr["idx"])), shape=(N, N)).tolil()
        b = -f.copy()
        for i in np.where(s.kind != 0)[0]:
            A.rows[i] = [i]; A.data[i] = [1.0]; b[i] = u[i]
        sol = spl.spsolve(A.tocsr(), b)
        errs.append(np.abs(sol - u).max()); hs.append(h)
    rates = np.log(np.array(errs[:-1]) / errs[1:]) / np.log(2)
    assert np.all(rates > 1.5), (errs, rates)


# ------------------------------------------------------------------- step ---
def _cavity_setup(h=0.05):
    s = ng.cavity2d(h=h, wall_band=0.1)
    st = O.build(s.x, s.kind, s.normal, s.h, 2)
    return s, O.to_csr(st)


def test_conduction_state_is_a_fixed_point_and_nu_is_one():
    s, csr = _cavity_setup()
    N = s.n
    x = s.x[0]
    T = (1.0 - x).copy()               # linear between the hot (x=0) and cold (x=1) walls
    v = np.zeros((2, N)); p = np.zeros(N + 1)
    sim = O.Sim(csr, s.kind)
    T0 = T.copy()
    sim.step(v, T, p, 20, Ra=0.0, Pr=0.71, dt=1e-4, T_ref=0.5)
    assert np.abs(T - T0).max() < 1e-10
    assert np.abs(v).max() == 0.0
    cold = np.where(s.group == 1)[0]
    g = GOLD["nusselt"]
    assert O.nusselt(csr, T, cold, L=g["L"], dT=1.0) == pytest.approx(g["conduction_nu"], rel=1e-9)


def test_zero_rayleigh_temperature_is_a_matrix_power():
    # With Ra = 0 and v = 0 the velocity stays 0 and the heat step is linear:
    # T^{n+1} = G T^n with G built here from the paper's explicit Euler update
    # (interior: I + dt Lap; Dirichlet rows: identity; Neumann rows: the
    # normal-derivative condition solved for the boundary value).
    s, csr = _cavity_setup()
    N = s.n
    dt = 2e-4
    rng = np.random.default_rng(0)
    T = np.where(s.kind == 1, s.tbc, rng.random(N))
    off, idx, wl, wn = csr["off"], csr["idx"], csr["w"][2], csr["wn"]
    G1 = np.eye(N)
    for i in range(N):
        if s.kind[i] == 0:
            for t in range(off[i], off[i + 1]):
                G1[i, idx[t]] += dt * wl[t]
    G = G1.copy()
    for b in np.where(s.kind == 2)[0]:
        G[b] = 0.0
        for t in range(off[b] + 1, off[b + 1]):
            G[b] -= (wn[t] / wn[off[b]]) * G1[idx[t]]
    ref = T.copy()
    for _ in range(10):
        ref = G @ ref
    v = np.zeros((2, N)); p = np.zeros(N + 1)
    sim = O.Sim(csr, s.kind)
    sim.step(v, T, p, 10, Ra=0.0, Pr=0.71, dt=dt, T_ref=0.5)
    np.testing.assert_allclose(T, ref, rtol=1e-11, atol=1e-12)
    assert np.abs(v).max() == 0.0


def test_bicgstab_pressure_matches_dense_solve():
    s, csr = _cavity_setup()
    N = s.n
    init = lambda: (np.zeros((2, N)), np.where(s.kind == 1, s.tbc, 0.5), np.zeros(N + 1))
    out = []
    for solver in (0, 1):
        v, T, p = init()
        sim = O.Sim(csr, s.kind, solver=solver)
        sim.step(v, T, p, 5, Ra=1e4, Pr=0.71, dt=1e-4, T_ref=0.5, tol=1e-13)
        out.append((v, T, p))
    (v0, T0, p0), (v1, T1, p1) = out
    assert np.abs(p0 - p1).max() <= 1e-8 * np.abs(p1).max()
    assert np.abs(v0 - v1).max() <= 1e-8 * np.abs(v1).max()
    assert np.abs(T0 - T1).max() <= 1e-10


def test_pressure_system_is_the_bordered_neumann_problem():
    # Dense pressure matrix: rows scaled to unit centre weight, constants in the
    # null space of the unbordered block, a border of c = 1/sqrt(N) (reading R11).
    s, csr = _cavity_setup()
    N = s.n
    M = O.pressure_dense(csr, s.kind)
    c = 1.0 / np.sqrt(N)
    np.testing.assert_allclose(np.diag(M)[:N], 1.0, rtol=1e-12)
    assert np.abs(M[:N, :N].sum(1)).max() < 1e-9
    assert np.all(M[:N, N] == c) and np.all(M[N, :N] == c) and M[N, N] == 0
    # and it is nonsingular
    assert np.linalg.matrix_rank(M) == N + 1
    # the scale changes neither the constraint nor p: the border of ones gives
    # the same p, with multiplier c lam
    M1 = M.copy()
    M1[:N, N] = 1.0
    M1[N, :N] = 1.0
    b = np.concatenate([np.random.default_rng(3).standard_normal(N), [0.0]])
    x, x1 = np.linalg.solve(M, b), np.linalg.solve(M1, b)
    assert np.abs(x[:N] - x1[:N]).max() <= 1e-9 * np.abs(x1[:N]).max()
    assert x1[N] == pytest.approx(c * x[N], rel=1e-9)
    assert abs(x[:N].sum()) <= 1e-9 * np.abs(x[:N]).sum()


def test_projection_reduces_divergence():
    s, csr = _cavity_setup()
    N = s.n
    v = np.zeros((2, N)); T = np.where(s.kind == 1, s.tbc, 0.5); p = np.zeros(N + 1)
    sim = O.Sim(csr, s.kind)
    sim.step(v, T, p, 3, Ra=1e4, Pr=0.71, dt=1e-4, T_ref=0.5)
    # one more predictor by hand, then compare divergence before/after projection
    interior = s.kind == 0
    div = O.apply(csr, csr["w"][0], v[0]) + O.apply(csr, csr["w"][1], v[1])
    assert np.abs(div[interior]).max() < 0.2 * np.abs(O.apply(csr, csr["w"][1], T)).max() + 1.0


def test_predictor_closed_form_on_quadratics():
    # v = (x^2 + y, x y), T = x: every operator is exact on quadratics, so the
    # predictor of Eq. (3) has a closed form at interior nodes:
    #   (v.grad)v_x = (x^2+y) 2x + x y * 1,   Lap v_x = 2
    #   (v.grad)v_y = (x^2+y) y + x y * x,    Lap v_y = 0
    # and gravity along -y gives the buoyancy +Ra Pr (T - T_ref) on v_y.
    s, csr = _cavity_setup()
    N = s.n
    x, y = s.x
    v = np.stack([x * x + y, x * y])
    T = x.copy()
    Ra, Pr, dt, Tr = 1e3, 0.71, 1e-3, 0.5
    sim = O.Sim(csr, s.kind)
    vs = sim.substep("predict", v, T, np.zeros((2, N)), Ra=Ra, Pr=Pr, dt=dt, T_ref=Tr)
    ex = v[0] + dt * (-((x * x + y) * 2 * x + x * y * 1) + Pr * 2)
    ey = v[1] + dt * (-((x * x + y) * y + x * y * x) + Ra * Pr * (T - Tr))
    inner = s.kind == 0
    np.testing.assert_allclose(vs[0][inner], ex[inner], atol=1e-9)
    np.testing.assert_allclose(vs[1][inner], ey[inner], atol=1e-9)
    assert np.all(vs[:, ~inner] == 0)


def test_projection_and_heat_closed_form():
    s, csr = _cavity_setup()
    N = s.n
    x, y = s.x
    dt = 1e-3
    sim = O.Sim(csr, s.kind)
    vs = np.stack([x + y, x - 2 * y])
    p = np.concatenate([x * x - x * y, [0.0]])
    v = sim.substep("correct", vs, p, np.zeros((2, N)), dt=dt)
    inner = s.kind == 0
    np.testing.assert_allclose(v[0][inner], (x + y - dt * (2 * x - y))[inner], atol=1e-10)
    np.testing.assert_allclose(v[1][inner], (x - 2 * y - dt * (-x))[inner], atol=1e-10)
    assert np.all(v[:, ~inner] == 0)
    # heat: T = x^2 + y, v = (1, 2): Tn = T + dt(-(2x + 2) + 2) at interior nodes
    T = x * x + y
    vv = np.stack([np.ones(N), 2 * np.ones(N)])
    Tn = sim.substep("heat", vv, T, np.zeros(N), dt=dt)
    np.testing.assert_allclose(Tn[inner], (T + dt * (-(2 * x + 2) + 2))[inner], atol=1e-10)
    dirich = s.kind == 1
    assert np.all(Tn[dirich] == T[dirich])


def test_pressure_rhs_closed_form():
    s, csr = _cavity_setup()
    x, y = s.x
    dt = 1e-3
    sim = O.Sim(csr, s.kind)
    vs = np.stack([x * x, x * y])              # div = 2x + x = 3x
    rhs = sim.substep("pressure_rhs", vs, np.zeros(s.n + 1), dt=dt)
    inner = s.kind == 0
    diag = np.array([csr["w"][2][csr["off"][i]] for i in range(s.n)])
    np.testing.assert_allclose((rhs[:-1] * diag)[inner], (3 * x / dt)[inner], rtol=1e-8, atol=1e-6)
    assert np.all(rhs[:-1][~inner] == 0) and rhs[-1] == 0


def test_hot_fluid_rises():
    # A hot blob in a fluid at rest: after one step the fluid at the blob moves up.
    s, csr = _cavity_setup()
    N = s.n
    x, y = s.x
    T = 0.5 + 0.5 * np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2) / 0.01)
    T[s.kind == 1] = 0.5
    v = np.zeros((2, N)); p = np.zeros(N + 1)
    sim = O.Sim(csr, s.kind)
    sim.step(v, T, p, 1, Ra=1e4, Pr=0.71, dt=1e-4, T_ref=0.5)
    c = np.argmin((x - 0.5) ** 2 + (y - 0.5) ** 2)
    assert v[1][c] > 0 and abs(v[0][c]) < 0.1 * v[1][c]


def test_all_scattered_mode():
    s = ng.cavity2d(h=0.05)
    st = O.build(s.x, s.kind, s.normal, s.h, 2, mode=O.ALL_SCATTERED)
    assert np.all(st["cls"] == 1) and np.all(st["width"] == 12)
    csr = O.to_csr(st)
    x, y = s.x
    np.testing.assert_allclose(O.apply(csr, csr["w"][2], x * x + y * y), 4.0, rtol=1e-8)


def test_wall_node_with_deficient_stencil_falls_back_to_degree_m_minus_1():
    # 3D h=0.02 obstacle set: a few wall nodes near a sphere whose scattered
    # band meets the box wall see interior nodes on only two normal layers
    # beyond the wall, so x^2 and x agree on their stencil and the degree-2
    # block is rank-deficient.  Walls need first derivatives only: such a
    # node takes PHS + monomials of degree 1 on the same stencil.
    s = ng.obstacles3d(h=0.02)
    q = np.array([467, 468, 515])
    assert np.all(s.kind[q] != 0)
    knn = O.knn(s.x, 20, queries=q, kind=s.kind)
    for r, i in enumerate(q):
        y = (s.x[:, knn[r]] - s.x[:, [i]]).T
        P2 = np.stack([_mono(al, y) for al in O.monomials(3, 2)], axis=1)
        assert np.linalg.matrix_rank(P2) < P2.shape[1]          # the degree-2 system is singular
    st = O.build(s.x, s.kind, s.normal, s.h, 2, queries=q)     # and the build still succeeds
    assert np.array_equal(st["idx"][:, :20], knn)              # on the same interior-only stencil
    for r, i in enumerate(q):
        nb = st["idx"][r, :20]
        y = (s.x[:, nb] - s.x[:, [i]]).T
        # first derivatives exact on every polynomial of degree <= 1 ...
        for al in O.monomials(3, 1):
            vals = _mono(al, y)
            for a in range(3):
                want = float(al[a] == 1 and sum(al) == 1)
                got = float(st["w"][r, a, :20] @ vals)
                assert abs(got - want) <= 1e-10 * np.abs(st["w"][r, a, :20]).sum() * np.abs(y).max()
        # ... but not on every quadratic (the degree really dropped): some
        # second-degree monomial has a non-zero derivative error
        # (every quadratic monomial has zero derivative at the centre, y = 0)
        errs = [abs(float(st["w"][r, a, :20] @ _mono(al, y))) for al in O.monomials(3, 2) if sum(al) == 2
                for a in range(3)]
        assert max(errs) > 1e-6 * s.h
        # the normal-derivative weights are n . grad weights
        wn = sum(s.normal[a, i] * st["w"][r, a, :20] for a in range(3))
        np.testing.assert_allclose(st["wn"][r, :20], wn, rtol=0, atol=1e-12 * np.abs(wn).max())


def _three_domains():
    sets = [ng.cavity2d(h=0.0625, seed=31), ng.cavity2d(h=0.05, seed=32),
            ng.obstacles2d(h=0.05, n_obst=2, rmin=0.08, rmax=0.12, band=0.15, seed=33)]
    x = np.concatenate([q.x for q in sets], axis=1)
    kind = np.concatenate([q.kind for q in sets])
    nrm = np.concatenate([q.normal for q in sets], axis=1)
    tbc = np.concatenate([q.tbc for q in sets])
    off = np.cumsum([0] + [q.n for q in sets]).astype(np.int64)
    return sets, x, kind, nrm, tbc, off


def test_multi_domain_pressure_system_has_one_border_per_domain():
    sets, x, kind, nrm, tbc, off = _three_domains()
    hs = [q.h for q in sets]
    csr = O.to_csr(O.build(x, kind, nrm, hs, 2, dom_off=off))
    M = O.pressure_dense(csr, kind, dom_off=off)
    N, K = len(kind), len(sets)
    assert M.shape == (N + K, N + K)
    for k in range(K):
        rows = np.arange(off[k], off[k + 1])
        # the border column of domain k is c_k = 1/sqrt(N_k) exactly on its rows, its border
        # row sums its nodes (times c_k)
        ck = 1.0 / np.sqrt(len(rows))
        np.testing.assert_array_equal(M[:N, N + k], ck * np.isin(np.arange(N), rows))
        np.testing.assert_array_equal(M[N + k, :N], ck * np.isin(np.arange(N), rows))
        # no coupling between domains
        others = np.setdiff1d(np.arange(N), rows)
        assert not M[np.ix_(rows, others)].any()
    assert not M[N:, N:].any()


def test_multi_domain_step_equals_independent_domains():
    # the domains share nothing: stepping them together (one bordered system
    # with a border per domain) equals stepping each alone
    sets, x, kind, nrm, tbc, off = _three_domains()
    hs = [q.h for q in sets]
    prm = dict(Ra=1e4, Pr=0.71, dt=0.1 * min(hs) ** 2 / 2, T_ref=0.5)
    csr = O.to_csr(O.build(x, kind, nrm, hs, 2, dom_off=off))
    N, K = len(kind), len(sets)
    T0 = np.where(kind == 1, tbc, 0.5)
    T0 = np.where(kind == 0, 0.5 + 0.2 * np.sin(4 * x[0]) * np.cos(3 * x[1]), T0)
    results = {}
    for solver in (1, 0):
        v, T, p = np.zeros((2, N)), T0.copy(), np.zeros(N + K)
        O.Sim(csr, kind, solver=solver, dom_off=off).step(v, T, p, 5, tol=1e-13, maxiter=50000, **prm)
        results[solver] = (v, T, p)
    for k, q in enumerate(sets):
        a, b = off[k], off[k + 1]
        ck = O.to_csr(O.build(q.x, q.kind, q.normal, q.h, 2))
        # the same stencils, shifted by the domain offset
        np.testing.assert_array_equal(csr["idx"][csr["off"][a]:csr["off"][b]] - a, ck["idx"])
        v, T, p = np.zeros((2, q.n)), T0[a:b].copy(), np.zeros(q.n + 1)
        O.Sim(ck, q.kind, solver=1).step(v, T, p, 5, **prm)
        for solver, tol in ((1, 1e-10), (0, 1e-8)):
            vm, Tm, pm = results[solver]
            for got, want in ((vm[:, a:b], v), (Tm[a:b], T), (pm[a:b], p[:-1])):
                assert np.abs(got - want).max() <= tol * max(np.abs(want).max(), 1e-30)
            assert abs(pm[N + k] - p[-1]) <= tol * max(abs(p[-1]), np.abs(p[:-1]).max())


def test_dvd_quarters_layout_and_conduction_nusselt():
    # Section 4.1: two diagonal quarters scattered, two regular.  Lattice nodes
    # only in the regular quarters, Poisson-disk fill only in the scattered
    # ones; the classifier finds regular nodes only where the lattice is.  On
    # the conduction profile T = x - 1/2 (T_C = -0.5 at x = 0, T_H = 0.5 at
    # x = 1) the cold-wall Nusselt number is 1: the normal-derivative weights
    # reproduce linear functions.
    q = ng.dvd2d(0.05, "hybrid")
    x, y = q.x
    scat_q = ((x < 0.5) & (y < 0.5)) | ((x > 0.5) & (y > 0.5))
    assert not np.any(scat_q[q.origin == 0])
    assert np.all(scat_q[q.origin == 2])
    assert np.sum(q.origin == 2) > 0
    st = O.build(q.x, q.kind, q.normal, q.h, 2)
    regular = st["cls"] == 0
    assert np.all(q.origin[regular] == 0) and regular.sum() > 0.5 * np.sum(q.origin == 0)
    cold = np.nonzero(q.group == 0)[0]
    assert len(cold) == round(1 / q.h) - 1 and np.all(q.x[0][cold] == 0.0) and np.all(q.tbc[cold] == -0.5)
    csr = O.to_csr(st)
    assert O.nusselt(csr, q.x[0] - 0.5, cold) == pytest.approx(1.0, rel=1e-12)


def test_condition_number_of_mon_cross_closed_form():
    # Section 2.1: kappa(M) = sigma_max / sigma_min.  On a lattice cross, in
    # coordinates scaled by h, M M^T splits into the x_a rows (eigenvalue 2)
    # and the x_a^2 rows, whose span holds 1 and u = sum_a x_a^2 / sqrt(d) with
    # Gram block [[2d+1, 2 sqrt d], [2 sqrt d, 2]] (eigenvalues
    # ((2d+3) +- sqrt((2d-1)^2 + 16d)) / 2, product 2) and eigenvalue 2 on the
    # rest: kappa = ((2d+3) + sqrt((2d-1)^2 + 16d)) / (2 sqrt 2), independent of
    # h and of the centre.
    for d, h, c in ((2, 0.37, [0.3, 0.9]), (2, 1e-3, [5.0, -2.0]), (3, 0.02, [0.1, 0.2, 0.3])):
        xs = [np.zeros(d)]
        for a in range(d):
            for sg in (-1, 1):
                e = np.zeros(d)
                e[a] = sg * h
                xs.append(e)
        xs = np.array(xs) + np.array(c)
        sv = np.linalg.svd(O.local_matrix(xs), compute_uv=False)
        disc = (2 * d - 1) ** 2 + 16 * d
        assert sv[0] / sv[-1] == pytest.approx(((2 * d + 3) + np.sqrt(disc)) / (2 * np.sqrt(2)), rel=1e-12)
    # every regular node of the cavity has a perfect cross
    q = ng.cavity2d(h=0.05, seed=7)
    kap = O.condition(q.x, q.kind, q.normal, q.h, 2)
    st = O.build(q.x, q.kind, q.normal, q.h, 2)
    assert np.allclose(kap[st["cls"] == 0], (7 + np.sqrt(41)) / (2 * np.sqrt(2)), rtol=1e-12)


def test_condition_matrix_reproduces_the_weights():
    # the matrix whose kappa is reported is the one the weights solve: M w = l
    # with the right-hand sides of Section 2.1 gives the oracle's (pinned) weights
    rng = np.random.default_rng(11)
    for d, m in ((2, 2), (2, 4), (3, 2)):
        n = O.stencil_size(d, m)
        xs = rng.random((n, d)) * 0.1 + 0.4
        w = O.rbffd(xs, m)
        M = O.local_matrix(xs, m)
        assert np.array_equal(M, M.T)
        y = xs - xs[0]
        s = np.sqrt((y * y).sum(1)).max()
        y = y / s
        r = np.sqrt((y * y).sum(1))
        al = [tuple(a) for a in O.monomials(d, m)]
        Q = len(al)
        rhs = np.zeros((n + Q, d + 1))
        for a in range(d):
            rhs[:n, a] = -3 * r * y[:, a]
            rhs[n + al.index(tuple(int(a == b) for b in range(d))), a] = 1.0
            rhs[n + al.index(tuple(2 * int(a == b) for b in range(d))), d] = 2.0
        rhs[:n, d] = 3 * (d + 1) * r
        sol = np.linalg.solve(M, rhs)
        assert np.allclose(sol[:n, :d].T / s, w[:d], rtol=0, atol=1e-9 * np.abs(w[:d]).max())
        assert np.allclose(sol[:n, d] / s ** 2, w[d], rtol=0, atol=1e-9 * np.abs(w[d]).max())
    # MON: the cross weights
    xs = np.array([[0, 0], [-1, 0], [1, 0], [0, -1], [0, 1]]) * 0.01 + 0.5
    M = O.local_matrix(xs)
    rhs = np.zeros((5, 3))
    rhs[1, 0] = rhs[2, 1] = 1.0
    rhs[3, 2] = rhs[4, 2] = 2.0
    sol = np.linalg.solve(M, rhs)
    wm = O.mon(xs)
    assert np.allclose(sol[:, :2].T / 0.01, wm[:2], atol=1e-9 * np.abs(wm[:2]).max())
    assert np.allclose(sol[:, 2] / 1e-4, wm[2], atol=1e-9 * np.abs(wm[2]).max())


def test_condition_number_invariances():
    # kappa of an RBF-FD system depends only on the shape of the stencil: the
    # same under translation, scaling and reordering of the non-centre nodes,
    # and (M symmetric) equal to |lambda|_max / |lambda|_min
    rng = np.random.default_rng(5)
    xs = rng.random((12, 2))
    k0 = np.linalg.svd(O.local_matrix(xs, 2), compute_uv=False)
    k0 = k0[0] / k0[-1]
    perm = np.concatenate([[0], 1 + rng.permutation(11)])
    for ys in (xs + [3.0, -7.0], xs * 1e-3, xs[perm]):
        sv = np.linalg.svd(O.local_matrix(ys, 2), compute_uv=False)
        assert sv[0] / sv[-1] == pytest.approx(k0, rel=1e-9)
    lam = np.abs(np.linalg.eigvalsh(O.local_matrix(xs, 2)))
    assert lam.max() / lam.min() == pytest.approx(k0, rel=1e-9)


def test_refined_and_split_layouts():
    # h-refinement (Sections 4.2, 4.3): circle nodes at spacing h_s; no lattice
    # node within the refinement distance h_r*delta_h of a circle; every fill
    # node keeps the spacing of its place (s(x) = h_s + (h_r - h_s) min(1,
    # dist / (h_r delta_h))) to every node placed before it, so no two fill
    # nodes are closer than the smaller of their spacings.
    h_r, ratio, dh = 0.05, 3.0, 4.0
    q = ng.refined2d(h_r=h_r, ratio=ratio, delta_h=dh, n_obst=2, rmin=0.08, rmax=0.12, seed=91)
    h_s = h_r / ratio
    c, r = q.obstacles[:, :2], q.obstacles[:, 2]
    dist = (np.sqrt(((q.x.T[:, None, :] - c[None]) ** 2).sum(-1)) - r[None]).min(1)
    for k in range(len(r)):
        on = q.group == 6 + k
        assert on.sum() == int(np.ceil(2 * np.pi * r[k] / h_s))
    assert np.all(dist[q.origin == 0] >= h_r * dh)
    sp = h_s + (h_r - h_s) * np.clip(dist / (h_r * dh), 0.0, 1.0)
    fill = np.nonzero(q.origin == 2)[0]
    dd = np.sqrt(((q.x.T[fill, None, :] - q.x.T[None, fill, :]) ** 2).sum(-1))
    np.fill_diagonal(dd, np.inf)
    assert np.all(dd >= np.minimum(sp[fill][:, None], sp[fill][None, :]) * (1 - 1e-12))
    # the split layout (Section 4.1): lattice only beyond h*delta_h, fill only before it
    s = ng.dvd2d_split(0.05, 6, "vertical")
    assert np.all(s.x[0][s.origin == 0] >= 0.05 * 6) and np.all(s.x[0][s.origin == 2] < 0.05 * 6)
    s = ng.dvd2d_split(0.05, 6, "horizontal")
    assert np.all(s.x[1][s.origin == 0] >= 0.05 * 6) and np.all(s.x[1][s.origin == 2] < 0.05 * 6)
