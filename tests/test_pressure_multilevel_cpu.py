"""Preconditioning the pressure solve: a CPU study on the oracle's pressure matrices.

The projection step (Section 3) solves a Poisson problem for the pressure with
Neumann rows at the walls and one zero-mean border row per domain.  Here that
bordered system, built from the oracle's FP64 stencils (rows divided by their
centre weight, as both solvers use it), is solved with scipy's BiCGSTAB: plain,
and preconditioned by a smoothed-aggregation V-cycle on the Laplacian block
with one of two restrictions:
  * Galerkin, R = P^T;
  * Petrov-Galerkin, R = ((I - w D^-1 A^T) P0)^T, the aggregates smoothed with
    the transposed operator (the RBF-FD Laplacian is not symmetric).
The tests hold the small-set figures the design notes quote.  Larger rows are
rerun with `python tests/test_pressure_multilevel_cpu.py obstacles 0.002 2`
(arguments: cavity|obstacles, h, m [, 1 for all-scattered] [, --ilu]).  Nothing here is
part of the GPU path.  CPU only.
"""
import json
import os
import sys

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))   # run as a script too
from oracle import oracle as O  # noqa: E402
from paper_2303_01760_amd import nodegen as ng  # noqa: E402


def bordered_matrix(csr, kind):
    """Laplacian block A [N, N] and the bordered system [[A, c1], [c1^T, 0]], c = 1/sqrt(N)."""
    N = len(csr["off"]) - 1
    rows = np.repeat(np.arange(N), np.diff(csr["off"]))
    vals = np.where(kind[rows] != 0, csr["wn"], csr["w"][csr["d"]])
    vals = vals / vals[csr["off"][:-1]][rows]
    A = sp.csr_matrix((vals, (rows, csr["idx"])), shape=(N, N))
    col = sp.csr_matrix(np.full((N, 1), 1.0 / np.sqrt(N)))
    return A, sp.bmat([[A, col], [col.T, None]], format="csr")


def aggregates(A, theta):
    """Greedy aggregation over the symmetrised strong couplings |a_ij| >= theta sqrt(|a_ii a_jj|)."""
    n = A.shape[0]
    dg = np.abs(A.diagonal())
    C = A.tocoo()
    keep = (C.row != C.col) & (np.abs(C.data) >= theta * np.sqrt(dg[C.row] * dg[C.col]))
    S = sp.csr_matrix((np.ones(keep.sum()), (C.row[keep], C.col[keep])), shape=(n, n))
    S = (S + S.T).tocsr()
    agg = np.full(n, -1, np.int64)
    na = 0
    for i in range(n):                       # seeds: nodes whose strong neighbours are all free
        nb = S.indices[S.indptr[i]:S.indptr[i + 1]]
        if agg[i] < 0 and np.all(agg[nb] < 0):
            agg[i] = na
            agg[nb] = na
            na += 1
    for i in range(n):                       # the rest join a neighbouring aggregate, else stand alone
        if agg[i] >= 0:
            continue
        nb = S.indices[S.indptr[i]:S.indptr[i + 1]]
        owners = agg[nb][agg[nb] >= 0]
        if len(owners):
            agg[i] = owners[0]
        else:
            agg[i] = na
            na += 1
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, na))


def hierarchy(A, petrov, theta=0.08, omega=4.0 / 3.0, coarsest=300):
    """Levels (A, P, R, diag) down to at most `coarsest` unknowns, and the coarsest solve."""
    levels = []
    while A.shape[0] > coarsest and len(levels) < 12:
        P0 = aggregates(A, theta)
        Dinv = sp.diags(1.0 / A.diagonal())
        v0 = np.random.default_rng(0).standard_normal(A.shape[0])     # a fixed start: the same levels every run
        rho = abs(spla.eigs(Dinv @ A, k=1, which="LM", v0=v0, return_eigenvectors=False, maxiter=200,
                            tol=1e-3)[0])
        P = (P0 - (omega / rho) * (Dinv @ (A @ P0))).tocsr()
        R = ((P0 - (omega / rho) * (Dinv @ (A.T @ P0))).T if petrov else P.T).tocsr()
        levels.append((A, P, R, A.diagonal()))
        A = (R @ A @ P).tocsr()
    # the coarsest operator keeps the constant null vector: a cut-off pseudo-inverse
    return levels, np.linalg.pinv(A.toarray(), rcond=1e-8), A


def vcycle(levels, coarse_inv, b, w=0.6):
    """One V-cycle, one damped-Jacobi sweep before and after each coarse correction."""
    def cycle(l, b):
        if l == len(levels):
            return coarse_inv @ b
        A, P, R, dg = levels[l]
        x = w * b / dg
        x = x + P @ cycle(l + 1, R @ (b - A @ x))
        return x + w * (b - A @ x) / dg
    return cycle(0, b)


def bicgstab_iterations(B, b, M=None, tol=1e-10, maxiter=20000):
    n = [0]
    x, info = spla.bicgstab(B, b, rtol=tol, atol=0.0, maxiter=maxiter, M=M,
                            callback=lambda _: n.__setitem__(0, n[0] + 1))
    return n[0], info, float(np.linalg.norm(b - B @ x) / np.linalg.norm(b))


def study(q, m=2, mode=O.HYBRID, plain=True, galerkin=True, ilu=False):
    """Iterations and fine-matvec work of each solver on the node set q (a smooth right-hand side);
    with ilu, also an incomplete LU held to the matrix's own fill (SuperLU, fill factor 1)."""
    csr = O.to_csr(O.build(q.x, q.kind, q.normal, q.h, m, mode=mode))
    A, B = bordered_matrix(csr, q.kind)
    N = A.shape[0]
    f = np.sin(3.1 * q.x[0] + 0.7) * np.cos(2.3 * q.x[1] - 0.4)
    f[q.kind != 0] = 0.0
    b = np.append(f, 0.0)
    out = dict(N=N)
    if plain:
        it, info, rel = bicgstab_iterations(B, b)
        out["plain"] = dict(iterations=it, info=info, relres=rel, work=2 * it)
    if ilu:
        try:
            lu = spla.spilu(B.tocsc(), drop_tol=0.0, fill_factor=1.0, permc_spec="NATURAL")
            it, info, rel = bicgstab_iterations(B, b, spla.LinearOperator(B.shape, lu.solve))
            out["ilu"] = dict(iterations=it, info=info, relres=rel)
        except RuntimeError as e:                 # a zero pivot
            out["ilu"] = dict(error=str(e))
    for name, petrov in (("galerkin", False), ("petrov_galerkin", True)):
        if name == "galerkin" and not galerkin:
            continue
        levels, cinv, Ac = hierarchy(A, petrov)
        complexity = (sum(L[0].nnz for L in levels) + Ac.nnz) / A.nnz

        def apply(v, levels=levels, cinv=cinv):
            return np.append(vcycle(levels, cinv, v[:N]), v[N])
        it, info, rel = bicgstab_iterations(B, b, spla.LinearOperator(B.shape, apply))
        # fine-matvec equivalents: 2 operator products and 2 V-cycles of 3 sweeps per level
        out[name] = dict(iterations=it, info=info, relres=rel, levels=len(levels) + 1,
                         work=it * (2 + 2 * 3 * complexity))
    return out


def test_petrov_galerkin_vcycle_count_stays_flat_as_the_cavity_is_refined():
    coarse = study(ng.dvd2d(0.02, "hybrid"))
    fine = study(ng.dvd2d(0.01, "hybrid"), galerkin=False)
    for r in (coarse, fine):
        assert r["plain"]["info"] == 0 and r["petrov_galerkin"]["info"] == 0
        assert r["petrov_galerkin"]["relres"] < 1e-9
    # plain BiCGSTAB grows like 1/h (272 -> 522 measured); the V-cycle's count does not (42 -> 47)
    assert fine["plain"]["iterations"] > 1.6 * coarse["plain"]["iterations"]
    assert fine["petrov_galerkin"]["iterations"] < 1.25 * coarse["petrov_galerkin"]["iterations"]
    assert fine["petrov_galerkin"]["iterations"] < 80
    assert fine["petrov_galerkin"]["work"] < 0.6 * fine["plain"]["work"]


def test_restriction_choice_on_the_obstacle_set():
    r = study(ng.obstacles2d(0.008))
    pg, g, pl = r["petrov_galerkin"], r["galerkin"], r["plain"]
    assert pg["info"] == 0 and pg["relres"] < 1e-9
    # measured 87 (Petrov-Galerkin), 198 (Galerkin), 819 (plain) iterations
    assert pg["iterations"] < 120
    assert g["iterations"] > 1.8 * pg["iterations"]
    assert pl["iterations"] > 6 * pg["iterations"]
    assert pg["work"] < 0.6 * pl["work"]


if __name__ == "__main__":
    kind, h, m = sys.argv[1], float(sys.argv[2]), int(sys.argv[3])
    mode = int(sys.argv[4]) if len(sys.argv) > 4 and not sys.argv[4].startswith("--") else O.HYBRID
    q = ng.dvd2d(h, "hybrid") if kind == "cavity" else ng.obstacles2d(h)
    print(json.dumps(dict(set=kind, h=h, m=m, mode=mode, **study(q, m, mode, ilu="--ilu" in sys.argv))))
