"""Python face of the FP64 CPU oracle (hsm_oracle.c).

TEST INFRASTRUCTURE ONLY: the plain reference the GPU library is checked
against.  Only tests, the smoke check and the benchmark's CPU-baseline leg use
it.  It never imports the GPU library, and the GPU library never imports it.

Every function follows a passage of the paper (Jancic, Rot, Kosec,
"Spatially-varying meshless approximation method for enhanced computational
efficiency"); the C source names the passage for each step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from math import comb

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsm_oracle.c")
_LIB = os.path.join(_HERE, "libhsm_oracle.so")
_lib = None

OK, E_INVALID, E_SINGULAR, E_DUPLICATE, E_NOT_CONVERGED, E_NONFINITE = 0, -1, -2, -3, -4, -5
HYBRID, ALL_SCATTERED = 0, 1

_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def build_library() -> str:
    """Compile the oracle (plain C, FP64, no contraction into FMA)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fPIC", "-shared",
           _SRC, "-o", _LIB, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class OracleParams(ctypes.Structure):
    _fields_ = [("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("dt", ctypes.c_double),
                ("T_ref", ctypes.c_double), ("tol", ctypes.c_double), ("maxiter", ctypes.c_int32),
                ("solver", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"oracle library not built: {_LIB} (run __graft_entry__.build())")
        L = ctypes.CDLL(_LIB)
        L.ora_knn.argtypes = [ctypes.c_int, _i64, _p, _p, _p, _i32, _i64, _p, ctypes.c_int, _p, _p]
        L.ora_classify.argtypes = [ctypes.c_int, _i64, _p, _p, _p, _i32, _p, _i64, _p, _p, _p]
        L.ora_dense_lu_solve.argtypes = [ctypes.c_int, _p, ctypes.c_int, _p, _p]
        L.ora_monomials.argtypes = [ctypes.c_int, ctypes.c_int, _p]
        L.ora_rbffd.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _p, _p]
        L.ora_mon.argtypes = [ctypes.c_int, _p, _p]
        L.ora_build.argtypes = [ctypes.c_int, _i64, _p, _p, _p, _p, _i32, _p, _p, _p, ctypes.c_int,
                                _i64, _p, ctypes.c_int, _p, _p, _p, _p, _p, _p]
        L.ora_weights_csr.argtypes = [ctypes.c_int, _i64, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _p]
        L.ora_apply.restype = None
        L.ora_apply.argtypes = [_i64, _p, _p, _p, _p, _p]
        L.ora_pressure_dense.argtypes = [_i64, _p, _p, _p, _p, _p, _i32, _p, _p]
        L.ora_sim_create.restype = _p
        L.ora_sim_create.argtypes = [ctypes.c_int, _i64, _p, _p, _p, _p, _p, _i32, _p, ctypes.c_int]
        L.ora_sim_destroy.restype = None
        L.ora_sim_destroy.argtypes = [_p]
        L.ora_sim_step.argtypes = [_p, ctypes.POINTER(OracleParams), ctypes.c_int, _p, _p, _p, _p]
        for f in ("ora_predict", "ora_pressure_rhs", "ora_correct", "ora_heat"):
            getattr(L, f).restype = None
        L.ora_predict.argtypes = [_p, ctypes.POINTER(OracleParams), _p, _p, _p]
        L.ora_pressure_rhs.argtypes = [_p, ctypes.POINTER(OracleParams), _p, _p]
        L.ora_correct.argtypes = [_p, ctypes.POINTER(OracleParams), _p, _p, _p]
        L.ora_heat.argtypes = [_p, ctypes.POINTER(OracleParams), _p, _p, _p]
        L.ora_nusselt.restype = ctypes.c_double
        L.ora_nusselt.argtypes = [_p, _p, _p, _p, _i64, _p, ctypes.c_double, ctypes.c_double]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def stencil_size(d: int, m: int) -> int:
    """n = 2 * C(m + d, m), the recommended RBF-FD stencil size (Section 1)."""
    return 2 * comb(m + d, m)


class OracleError(RuntimeError):
    def __init__(self, code, node=-1):
        super().__init__(f"oracle error {code} (node {node})")
        self.code, self.node = code, node


def knn(x, k, dom_off=None, queries=None, kind=None):
    """k nearest nodes of each query within its domain, ordered by (d2, index).

    With kind given, a boundary query (kind != 0) draws from itself and the
    interior nodes only."""
    x = _c(x, np.float64)
    d, N = x.shape
    dom_off = _c(dom_off if dom_off is not None else [0, N], np.int64)
    q = None if queries is None else _c(queries, np.int64)
    nq = N if q is None else len(q)
    out = np.empty((nq, k), np.int32)
    bad = np.array([-1], np.int64)
    kd = None if kind is None else _c(kind, np.uint8)
    rc = lib().ora_knn(d, N, _ptr(x), _ptr(kd), _ptr(dom_off), len(dom_off) - 1, nq, _ptr(q), k, _ptr(out), _ptr(bad))
    if rc:
        raise OracleError(rc, int(bad[0]))
    return out


def classify(x, kind, h, dom_off=None, queries=None):
    """Regular (0) / scattered (1) per node and the axis cross of regular nodes."""
    x = _c(x, np.float64)
    d, N = x.shape
    dom_off = _c(dom_off if dom_off is not None else [0, N], np.int64)
    hd = _c(np.broadcast_to(np.asarray(h, np.float64), (len(dom_off) - 1,)), np.float64)
    q = None if queries is None else _c(queries, np.int64)
    nq = N if q is None else len(q)
    cls = np.empty(nq, np.uint8)
    cross = np.empty((nq, 2 * d + 1), np.int32)
    rc = lib().ora_classify(d, N, _ptr(x), _ptr(_c(kind, np.uint8)), _ptr(dom_off), len(dom_off) - 1,
                            _ptr(hd), nq, _ptr(q), _ptr(cls), _ptr(cross))
    if rc:
        raise OracleError(rc)
    return cls, cross


def dense_lu_solve(a, b):
    a = np.array(a, np.float64, order="C")
    b = np.array(b, np.float64, order="C")
    squeeze = b.ndim == 1
    if squeeze:
        b = b[:, None].copy()
    S, R = b.shape
    x = np.empty((S, R), np.float64)
    rc = lib().ora_dense_lu_solve(S, _ptr(a), R, _ptr(b), _ptr(x))
    if rc:
        raise OracleError(rc)
    return x[:, 0] if squeeze else x


def monomials(d, m):
    al = np.zeros((256, 3), np.int32)
    q = lib().ora_monomials(d, m, _ptr(al))
    return al[:q, :d].copy()


def rbffd(xs, m):
    """RBF-FD weights [d+1, n] (d/dx_a ..., Laplacian) for stencil positions xs [n, d], centre first."""
    xs = _c(xs, np.float64)
    n, d = xs.shape
    w = np.empty((d + 1, n), np.float64)
    rc = lib().ora_rbffd(d, m, n, _ptr(xs), _ptr(w))
    if rc:
        raise OracleError(rc)
    return w


def mon(xs):
    """MON weights [d+1, 2d+1] for the cross positions xs [2d+1, d], centre first."""
    xs = _c(xs, np.float64)
    n, d = xs.shape
    w = np.empty((d + 1, n), np.float64)
    rc = lib().ora_mon(d, _ptr(xs), _ptr(w))
    if rc:
        raise OracleError(rc)
    return w


def build(x, kind, normal, h, m, mode=HYBRID, dom_off=None, queries=None, n=None):
    """Class, stencil and weights of each query node (all nodes if queries is None).

    h, m, n may be scalars or per-domain sequences.  Returns a dict of padded
    arrays: cls [nq], width [nq], idx [nq, maxw], w [nq, d+1, maxw], wn [nq, maxw].
    """
    x = _c(x, np.float64)
    d, N = x.shape
    dom_off = _c(dom_off if dom_off is not None else [0, N], np.int64)
    nd = len(dom_off) - 1
    hd = _c(np.broadcast_to(np.asarray(h, np.float64), (nd,)), np.float64)
    md = _c(np.broadcast_to(np.asarray(m, np.int32), (nd,)), np.int32)
    if n is None:
        nn = np.array([stencil_size(d, int(mm)) for mm in md], np.int32)
    else:
        nn = _c(np.broadcast_to(np.asarray(n, np.int32), (nd,)), np.int32)
    maxw = int(max(int(nn.max()), 2 * d + 1))
    q = None if queries is None else _c(queries, np.int64)
    nq = N if q is None else len(q)
    cls = np.empty(nq, np.uint8)
    width = np.empty(nq, np.int32)
    idx = np.empty((nq, maxw), np.int32)
    w = np.empty((nq, d + 1, maxw), np.float64)
    wn = np.empty((nq, maxw), np.float64)
    bad = np.array([-1], np.int64)
    rc = lib().ora_build(d, N, _ptr(x), _ptr(_c(kind, np.uint8)), _ptr(_c(normal, np.float64)),
                         _ptr(dom_off), nd, _ptr(hd), _ptr(md), _ptr(nn), int(mode), nq, _ptr(q), maxw,
                         _ptr(cls), _ptr(width), _ptr(idx), _ptr(w), _ptr(wn), _ptr(bad))
    if rc:
        raise OracleError(rc, int(bad[0]))
    return dict(cls=cls, width=width, idx=idx, w=w, wn=wn, d=d)


def local_matrix(xs, m=None):
    """The matrix M of a node's local system M w = l (Section 2.1) for stencil
    positions xs [n, d], centre first, in the solve's local coordinates
    y = (x - x_c) / s, s = max_j |x_j - x_c| (reading R5).  m=None: the MON
    matrix of a regular node (rows: the basis 1, y_a, y_a^2; columns: the
    cross nodes).  Otherwise the RBF-FD matrix [[A, P], [P^T, 0]] with
    A_jl = |y_j - y_l|^3 and P_ja = y_j^alpha for every monomial of degree
    <= m."""
    xs = np.asarray(xs, np.float64)
    n, d = xs.shape
    y = xs - xs[0]
    s = np.sqrt((y * y).sum(axis=1)).max()
    y = y / s
    if m is None:
        return np.vstack([np.ones(n), y.T, (y * y).T])
    al = monomials(d, m)
    P = np.stack([np.prod(y ** a, axis=1) for a in al], axis=1)
    A = np.sqrt(((y[:, None, :] - y[None, :, :]) ** 2).sum(axis=2)) ** 3
    Q = P.shape[1]
    return np.block([[A, P], [P.T, np.zeros((Q, Q))]])


def condition(x, kind, normal, h, m, mode=HYBRID, dom_off=None, queries=None, n=None):
    """kappa(M) = |M|_2 |M^-1|_2 = sigma_max / sigma_min of each query node's
    local system (Section 2.1, Fig. 2), singular values by LAPACK.  The system
    is the one solved for the node's weights: MON at regular nodes, RBF-FD at
    scattered ones, with degree m-1 at a wall node whose degree-m system is
    singular (reading R17)."""
    x = np.asarray(x, np.float64)
    d, N = x.shape
    st = build(x, kind, normal, h, m, mode=mode, dom_off=dom_off, queries=queries, n=n)
    q = np.arange(N) if queries is None else np.asarray(queries, np.int64)
    off = np.asarray(dom_off if dom_off is not None else [0, N], np.int64)
    md = np.broadcast_to(np.asarray(m, np.int64), (len(off) - 1,))
    kappa = np.empty(len(q))
    for k, i in enumerate(q):
        xs = x[:, st["idx"][k, :st["width"][k]]].T
        if st["cls"][k] == 0:
            M = local_matrix(xs)
        else:
            mm = int(md[np.searchsorted(off, i, side="right") - 1])
            try:
                rbffd(xs, mm)
            except OracleError as e:
                if e.code != E_SINGULAR or kind[i] == 0 or mm < 2:
                    raise
                mm -= 1
            M = local_matrix(xs, mm)
        sv = np.linalg.svd(M, compute_uv=False)
        kappa[k] = sv[0] / sv[-1] if sv[-1] > 0 else np.inf
    return kappa


def to_csr(st):
    """Padded per-node stencils -> CSR (off, idx, w[d+1], wn)."""
    width = st["width"].astype(np.int64)
    off = np.zeros(len(width) + 1, np.int64)
    np.cumsum(width, out=off[1:])
    mask = np.arange(st["idx"].shape[1])[None, :] < width[:, None]
    idx = st["idx"][mask].astype(np.int32)
    d = st["d"]
    w = np.stack([st["w"][:, r, :][mask] for r in range(d + 1)])
    wn = st["wn"][mask]
    return dict(off=off, idx=idx, w=w, wn=wn, d=d, cls=st["cls"], width=st["width"])


def weights_csr(x, kind, csr, m, nodes=None):
    """The local solves alone for the stencils of a CSR set (no neighbour
    search): weights [d+1, nnz] of the nodes `nodes` (default 0..n-1), MON
    where csr["cls"] is 0, RBF-FD of degree m (scalar or per stencil)
    elsewhere.  Same arithmetic as build()."""
    x = _c(x, np.float64)
    d, N = x.shape
    off = _c(csr["off"], np.int64)
    ns = len(off) - 1
    nodes = _c(np.arange(ns) if nodes is None else nodes, np.int64)
    mm = _c(np.broadcast_to(np.asarray(m, np.int32), (ns,)), np.int32)
    w = np.empty((d + 1, int(off[-1])), np.float64)
    bad = np.array([-1], np.int64)
    rc = lib().ora_weights_csr(d, N, _ptr(x), _ptr(_c(kind, np.uint8)), ns, _ptr(nodes), _ptr(off),
                               _ptr(_c(csr["idx"], np.int32)), _ptr(_c(csr["cls"], np.uint8)), _ptr(mm), _ptr(w),
                               _ptr(bad))
    if rc:
        raise OracleError(rc, int(bad[0]))
    return w


def apply(csr, wrow, u):
    """Eq. (1) at every node: out_i = sum_j w_ij u_j (stencil order)."""
    u = _c(u, np.float64)
    N = len(csr["off"]) - 1
    out = np.empty(N, np.float64)
    lib().ora_apply(N, _ptr(csr["off"]), _ptr(csr["idx"]), _ptr(_c(wrow, np.float64)), _ptr(u), _ptr(out))
    return out


def pressure_dense(csr, kind, dom_off=None):
    """The bordered pressure matrix [(N+K)^2]: one border row/column per domain."""
    N = len(csr["off"]) - 1
    dom_off = _c(dom_off if dom_off is not None else [0, N], np.int64)
    K = len(dom_off) - 1
    M = np.empty((N + K, N + K), np.float64)
    d = csr["d"]
    lib().ora_pressure_dense(N, _ptr(csr["off"]), _ptr(csr["idx"]), _ptr(_c(csr["w"][d], np.float64)),
                             _ptr(_c(csr["wn"], np.float64)), _ptr(_c(kind, np.uint8)), K, _ptr(dom_off), _ptr(M))
    return M


class Sim:
    """Explicit Euler Boussinesq stepping with Chorin projection (Section 3)."""

    def __init__(self, csr, kind, solver=0, dom_off=None):
        self.csr = csr
        self.kind = _c(kind, np.uint8)
        d = csr["d"]
        self._w = [_c(csr["w"][a], np.float64) for a in range(d + 1)]
        arr = (ctypes.c_void_p * 4)(*[w.ctypes.data for w in self._w], *([None] * (3 - d)))
        self._wn = _c(csr["wn"], np.float64)
        N = len(csr["off"]) - 1
        self._dom_off = _c(dom_off if dom_off is not None else [0, N], np.int64)
        self.N, self.d, self.K = N, d, len(self._dom_off) - 1
        self.h = lib().ora_sim_create(d, N, _ptr(csr["off"]), _ptr(csr["idx"]), arr, _ptr(self._wn),
                                      _ptr(self.kind), self.K, _ptr(self._dom_off), int(solver))
        if not self.h:
            raise OracleError(E_INVALID)

    def step(self, v, T, p, nsteps, Ra, Pr, dt, T_ref, tol=1e-12, maxiter=20000):
        """Advance v [d,N], T [N], p [N+K] in place by nsteps; returns Krylov iterations per step."""
        for a, shape in ((v, (self.d, self.N)), (T, (self.N,)), (p, (self.N + self.K,))):
            assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape == shape
        prm = OracleParams(Ra, Pr, dt, T_ref, tol, maxiter, 0)
        its = np.zeros(nsteps, np.int32)
        rc = lib().ora_sim_step(self.h, ctypes.byref(prm), nsteps, _ptr(v), _ptr(T), _ptr(p), _ptr(its))
        if rc:
            raise OracleError(rc)
        return its

    def substep(self, name, *arrays, Ra=0.0, Pr=0.71, dt=1e-4, T_ref=0.5):
        """Run one sub-step (predict, pressure_rhs, correct, heat) on given arrays; the last one is written."""
        prm = OracleParams(Ra, Pr, dt, T_ref, 0.0, 0, 0)
        arrs = [np.ascontiguousarray(a, np.float64) for a in arrays]
        getattr(lib(), "ora_" + name)(self.h, ctypes.byref(prm), *[_ptr(a) for a in arrs])
        return arrs[-1]

    def close(self):
        if self.h:
            lib().ora_sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nusselt(csr, T, nodes, L=1.0, dT=1.0):
    nodes = _c(nodes, np.int64)
    return lib().ora_nusselt(_ptr(csr["off"]), _ptr(csr["idx"]), _ptr(_c(csr["wn"], np.float64)),
                             _ptr(_c(T, np.float64)), len(nodes), _ptr(nodes), L, dT)
