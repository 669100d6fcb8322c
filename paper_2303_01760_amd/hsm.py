"""Python binding of libhsm.so (include/hsm.h), same names, argument marshalling only.

Every computation runs in the library's HIP kernels; torch supplies device
memory and the current stream.  There is no fallback: if the library is not
built or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsm.so")

OK, E_INVALID, E_SINGULAR, E_DUPLICATE_NODE, E_NOT_CONVERGED, E_NONFINITE, E_HIP, E_OOM, E_AMBIGUOUS = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
OP_DX, OP_DY, OP_DZ, OP_LAP, OP_DN = 1, 2, 4, 8, 16
F64, F32, F32_COMP = 0, 1, 2
MODE_HYBRID, MODE_ALL_SCATTERED = 0, 1
TO_INTERNAL, TO_CALLER = 0, 1

_p = ctypes.c_void_p


class NodeSetC(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n_domains", ctypes.c_int32),
                ("host_domain_offsets", _p), ("x", _p), ("kind", _p), ("normal", _p),
                ("host_h_regular", _p), ("host_m", _p), ("host_n", _p), ("tile_log2", ctypes.c_int32),
                ("solve_groups", ctypes.c_int32)]


class StencilsInfoC(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("mode", ctypes.c_int32), ("n_domains", ctypes.c_int32),
                ("n_buckets", ctypes.c_int32), ("n_nodes", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("n_regular", ctypes.c_int64), ("n_scattered", ctypes.c_int64), ("n_boundary", ctypes.c_int64),
                ("n_wall_fallback", ctypes.c_int64), ("bucket_width", ctypes.c_int32 * 16), ("bucket_type", ctypes.c_int32 * 16),
                ("bucket_count", ctypes.c_int64 * 16), ("build_ms", ctypes.c_double * 4),
                ("bucket_solve_ms", ctypes.c_double * 16)]


class SimParamsC(ctypes.Structure):
    _fields_ = [("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("dt", ctypes.c_double),
                ("T_ref", ctypes.c_double), ("krylov_tol", ctypes.c_double), ("krylov_maxiter", ctypes.c_int32),
                ("field_dtype", ctypes.c_int32), ("krylov_chunk", ctypes.c_int32), ("launch_mode", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("reduce_mode", ctypes.c_int32), ("block_nodes", ctypes.c_int32),
                ("gather_chunk", ctypes.c_int32), ("xcd_order", ctypes.c_int32), ("lattice_rows", ctypes.c_int32),
                ("wide_lanes", ctypes.c_int32)]


class SimStatsC(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("krylov_iters_total", ctypes.c_int64),
                ("krylov_iters_last", ctypes.c_int32), ("status", ctypes.c_int32),
                ("last_relres", ctypes.c_double), ("node_applies", ctypes.c_int64),
                ("krylov_node_matvecs", ctypes.c_int64), ("krylov_reduced_batches", ctypes.c_int64)]


_lib = None

# every symbol include/hsm.h declares
SYMBOLS = ["hsm_build_stencils", "hsm_stencils_get_info", "hsm_stencils_export", "hsm_permute",
           "hsm_apply_operator", "hsm_apply_node_count", "hsm_sim_create", "hsm_step", "hsm_sim_get_stats",
           "hsm_sim_read", "hsm_sim_destroy", "hsm_stencils_destroy", "hsm_last_error", "hsm_last_error_node",
           "hsm_version", "hsm_sim_phase_times", "hsm_sim_sizes", "hsm_stream_copy", "hsm_stencils_condition",
           "hsm_apply_operator_buckets", "hsm_stencils_export_noalloc"]
PHASES = ["pre", "krylov_iter", "post", "krylov_batch"]


def lib():
    """Load libhsm.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int32
        L.hsm_build_stencils.restype = st
        L.hsm_build_stencils.argtypes = [ctypes.POINTER(NodeSetC), ctypes.c_int32, _p, ctypes.POINTER(_p)]
        L.hsm_stencils_get_info.restype = st
        L.hsm_stencils_get_info.argtypes = [_p, ctypes.POINTER(StencilsInfoC)]
        L.hsm_stencils_export.restype = st
        L.hsm_stencils_export.argtypes = [_p, _p, _p, _p, _p, _p]
        L.hsm_stencils_export_noalloc.restype = st
        L.hsm_stencils_export_noalloc.argtypes = [_p, _p, _p, _p, _p, _p]
        L.hsm_permute.restype = st
        L.hsm_permute.argtypes = [_p, ctypes.c_int32, ctypes.c_int32, _p, _p, _p]
        L.hsm_apply_operator.restype = st
        L.hsm_apply_operator.argtypes = [_p, ctypes.c_uint32, ctypes.c_int32, _p, _p, _p]
        L.hsm_apply_node_count.restype = ctypes.c_int64
        L.hsm_apply_node_count.argtypes = [_p, ctypes.c_uint32]
        L.hsm_sim_create.restype = st
        L.hsm_sim_create.argtypes = [_p, ctypes.POINTER(SimParamsC), _p, _p, _p, _p, ctypes.POINTER(_p)]
        L.hsm_step.restype = st
        L.hsm_step.argtypes = [_p, ctypes.c_int32, _p]
        L.hsm_sim_get_stats.restype = st
        L.hsm_sim_get_stats.argtypes = [_p, ctypes.POINTER(SimStatsC)]
        L.hsm_sim_read.restype = st
        L.hsm_sim_read.argtypes = [_p, _p, _p, _p, _p]
        L.hsm_sim_destroy.restype = None
        L.hsm_sim_destroy.argtypes = [_p]
        L.hsm_stencils_destroy.restype = None
        L.hsm_stencils_destroy.argtypes = [_p]
        L.hsm_last_error.restype = ctypes.c_char_p
        L.hsm_last_error.argtypes = []
        L.hsm_last_error_node.restype = ctypes.c_int64
        L.hsm_last_error_node.argtypes = []
        L.hsm_sim_phase_times.restype = st
        L.hsm_sim_phase_times.argtypes = [_p, _p, _p]
        L.hsm_sim_sizes.restype = st
        L.hsm_sim_sizes.argtypes = [_p, _p]
        L.hsm_stream_copy.restype = st
        L.hsm_stream_copy.argtypes = [_p, _p, ctypes.c_int64, _p]
        L.hsm_stencils_condition.restype = st
        L.hsm_stencils_condition.argtypes = [_p, _p, _p]
        L.hsm_apply_operator_buckets.restype = st
        L.hsm_apply_operator_buckets.argtypes = [_p, ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint32, _p, _p, _p]
        L.hsm_version.restype = ctypes.c_char_p
        L.hsm_version.argtypes = []
        _lib = L
    return _lib


class HsmError(RuntimeError):
    def __init__(self, code: int, msg: str, node: int):
        super().__init__(msg)
        self.code, self.node = code, node


def _check(rc: int):
    if rc != OK:
        L = lib()
        raise HsmError(rc, L.hsm_last_error().decode(), int(L.hsm_last_error_node()))


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t: torch.Tensor, dtype=None):
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    if dtype is not None:
        assert t.dtype == dtype, f"expected {dtype}, got {t.dtype}"
    return ctypes.c_void_p(t.data_ptr())


class Stencils:
    """Handle of a built stencil set (hsm_stencils)."""

    def __init__(self, handle, d, n):
        self._h = handle
        self.d, self.n = d, n

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        o = StencilsInfoC()
        _check(lib().hsm_stencils_get_info(self._h, ctypes.byref(o)))
        nb = o.n_buckets
        return dict(d=o.d, mode=o.mode, n_domains=o.n_domains, n_nodes=o.n_nodes, nnz=o.nnz,
                    n_regular=o.n_regular, n_scattered=o.n_scattered, n_boundary=o.n_boundary,
                    n_wall_fallback=o.n_wall_fallback,
                    buckets=[(o.bucket_type[k], o.bucket_width[k], o.bucket_count[k]) for k in range(nb)],
                    build_ms=list(o.build_ms), bucket_solve_ms=list(o.bucket_solve_ms[:nb]))

    def export(self, stream=None, noalloc: bool = False) -> dict:
        """Classes, CSR stencils (caller numbering) and weights [d+2, nnz] as numpy arrays.
        noalloc: through hsm_stencils_export_noalloc (device temporaries from the library's fixed array)."""
        info = self.info()
        N, nnz, d = info["n_nodes"], info["nnz"], info["d"]
        cls = np.empty(N, np.uint8)
        off = np.empty(N + 1, np.int64)
        idx = np.empty(max(nnz, 1), np.int32)
        w = np.empty((d + 2, max(nnz, 1)), np.float64)
        fn = lib().hsm_stencils_export_noalloc if noalloc else lib().hsm_stencils_export
        _check(fn(self._h, cls.ctypes.data, off.ctypes.data, idx.ctypes.data, w.ctypes.data, _stream(stream)))
        return dict(cls=cls, off=off, idx=idx[:nnz], w=w[:, :nnz], d=d)

    def permute(self, src: torch.Tensor, direction: int, stream=None) -> torch.Tensor:
        dt = F64 if src.dtype == torch.float64 else F32
        dst = torch.empty_like(src)
        _check(lib().hsm_permute(self._h, direction, dt, _dptr(src), _dptr(dst), _stream(stream)))
        return dst

    def to_internal(self, t, stream=None):
        return self.permute(t, TO_INTERNAL, stream)

    def to_caller(self, t, stream=None):
        return self.permute(t, TO_CALLER, stream)

    def apply(self, u: torch.Tensor, op_mask: int, dtype: int = F64, out=None, stream=None) -> torch.Tensor:
        """Eq. (1) for every operator in op_mask; u and the result are in internal order."""
        nops = bin(op_mask & 31).count("1")
        tdt = torch.float64 if dtype == F64 else torch.float32
        if out is None:
            out = torch.empty((nops, self.n), dtype=tdt, device=u.device)
        apply_operator(self, op_mask, dtype, u, out, stream)
        return out

    def condition(self, stream=None) -> torch.Tensor:
        """hsm_stencils_condition: kappa(M) of every node's local system, caller order."""
        out = torch.empty(self.n, dtype=torch.float64, device=torch.device("cuda"))
        _check(lib().hsm_stencils_condition(self._h, _dptr(out), _stream(stream)))
        return out

    def apply_buckets(self, u: torch.Tensor, op_mask: int, bucket_mask: int, dtype: int = F64, out=None,
                      stream=None) -> torch.Tensor:
        """hsm_apply_operator_buckets: Eq. (1) on the buckets in bucket_mask only (internal order)."""
        nops = bin(op_mask & 31).count("1")
        tdt = torch.float64 if dtype == F64 else torch.float32
        if out is None:
            out = torch.zeros((nops, self.n), dtype=tdt, device=u.device)
        _check(lib().hsm_apply_operator_buckets(self._h, int(op_mask), int(dtype), int(bucket_mask), _dptr(u),
                                                _dptr(out), _stream(stream)))
        return out

    def node_count(self, op_mask: int) -> int:
        return int(lib().hsm_apply_node_count(self._h, op_mask))

    def close(self):
        if self._h:
            lib().hsm_stencils_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_stencils(x: torch.Tensor, kind: torch.Tensor, normal: torch.Tensor, h, m, mode=MODE_HYBRID,
                   domain_offsets=None, n=None, tile_log2=0, solve_groups=0, stream=None) -> Stencils:
    """hsm_build_stencils on device tensors x [d,N] f64, kind [N] u8, normal [d,N] f64."""
    d, N = x.shape
    offs = np.asarray(domain_offsets if domain_offsets is not None else [0, N], np.int64)
    nd = len(offs) - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, np.float64), (nd,)))
    ms = np.ascontiguousarray(np.broadcast_to(np.asarray(m, np.int32), (nd,)))
    ns_ = None if n is None else np.ascontiguousarray(np.broadcast_to(np.asarray(n, np.int32), (nd,)))
    c = NodeSetC(d, nd, offs.ctypes.data, _dptr(x, torch.float64), _dptr(kind, torch.uint8),
                 _dptr(normal, torch.float64), hs.ctypes.data, ms.ctypes.data,
                 None if ns_ is None else ns_.ctypes.data, int(tile_log2), int(solve_groups))
    h_out = _p()
    _check(lib().hsm_build_stencils(ctypes.byref(c), int(mode), _stream(stream), ctypes.byref(h_out)))
    return Stencils(h_out.value, d, N)


def stream_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """hsm_stream_copy: plain device copy (measurement aid)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= nbytes
    _check(lib().hsm_stream_copy(_dptr(src), _dptr(dst), nbytes, _stream(stream)))


def apply_operator(st: Stencils, op_mask: int, dtype: int, u: torch.Tensor, out: torch.Tensor, stream=None):
    _check(lib().hsm_apply_operator(st.handle, int(op_mask), int(dtype), _dptr(u), _dptr(out), _stream(stream)))


class Sim:
    """hsm_sim: explicit Boussinesq stepping on a stencil set."""

    def __init__(self, st: Stencils, v: torch.Tensor, T: torch.Tensor, p=None, *, Ra, Pr, dt, T_ref,
                 krylov_tol=1e-12, krylov_maxiter=20000, field_dtype=F64, krylov_chunk=0, launch_mode=0,
                 profile=0, reduce_mode=0, block_nodes=0, gather_chunk=0, xcd_order=0, lattice_rows=0,
                 wide_lanes=0, stream=None):
        self.st = st
        prm = SimParamsC(Ra, Pr, dt, T_ref, krylov_tol, krylov_maxiter, field_dtype, krylov_chunk, launch_mode,
                         profile, reduce_mode, block_nodes, gather_chunk, xcd_order, lattice_rows, wide_lanes)
        h = _p()
        _check(lib().hsm_sim_create(st.handle, ctypes.byref(prm), _dptr(v, torch.float64), _dptr(T, torch.float64),
                                    None if p is None else _dptr(p, torch.float64), _stream(stream),
                                    ctypes.byref(h)))
        self._h = h.value

    def step(self, nsteps: int, stream=None):
        _check(lib().hsm_step(self._h, int(nsteps), _stream(stream)))

    def stats(self) -> dict:
        o = SimStatsC()
        rc = lib().hsm_sim_get_stats(self._h, ctypes.byref(o))
        d = dict(steps=o.steps, krylov_iters_total=o.krylov_iters_total, krylov_iters_last=o.krylov_iters_last,
                 status=o.status, last_relres=o.last_relres, node_applies=o.node_applies,
                 krylov_node_matvecs=o.krylov_node_matvecs, krylov_reduced_batches=o.krylov_reduced_batches)
        if rc not in (OK, E_NONFINITE, E_NOT_CONVERGED):
            _check(rc)
        return d

    def phase_times(self) -> dict:
        """Mean device ms and sample count of each timed phase (profile mode)."""
        ms = np.zeros(len(PHASES))
        cnt = np.zeros(len(PHASES), np.int64)
        _check(lib().hsm_sim_phase_times(self._h, ms.ctypes.data, cnt.ctypes.data))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PHASES)}

    def sizes(self) -> dict:
        info = np.zeros(6, np.int64)
        _check(lib().hsm_sim_sizes(self._h, info.ctypes.data))
        return dict(N=int(info[0]), nnz=int(info[1]), n_interior=int(info[2]), n_neumann=int(info[3]),
                    n_shared_rows=int(info[4]), nnz_shared_rows=int(info[5]))

    def read(self, stream=None):
        d, N = self.st.d, self.st.n
        dev = torch.device("cuda")
        v = torch.empty((d, N), dtype=torch.float64, device=dev)
        T = torch.empty(N, dtype=torch.float64, device=dev)
        p = torch.empty(N, dtype=torch.float64, device=dev)
        _check(lib().hsm_sim_read(self._h, _dptr(v), _dptr(T), _dptr(p), _stream(stream)))
        return v, T, p

    def close(self):
        if self._h:
            lib().hsm_sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
