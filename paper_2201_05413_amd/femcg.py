"""ctypes binding of libfemcg.so (argument marshalling only).

Every call has the name and meaning of the C function declared in
include/femcg.h.  Device arrays are torch CUDA tensors (float64, contiguous,
row-major [n][k]); streams are torch.cuda streams.  All arithmetic runs in the
library's HIP kernels; this module never computes anything itself, and it
raises if the library is not built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfemcg.so")

FEMCG_OK = 0
FEMCG_WARN_MAXITER = 1
FEMCG_EINVAL = -1
FEMCG_EMESH = -2
FEMCG_ENOMEM = -3
FEMCG_EBREAKDOWN = -4
FEMCG_EUNSUPPORTED = -5
FEMCG_EDEVICE = -6
FEMCG_EADMIT = -7
FEMCG_MAX_K = 64

FEM_FORMAT_CSR = 0
FEM_FORMAT_SELL = 1
FEM_FORMAT_AUTO = 2
FEM_ORDER_SFC = 0x10
FEM_ASSEMBLE_DEVICE = 0x100
FEM_ASSEMBLE_HOST_ONLY = 0x200
PCG_FP64 = 0
PCG_MIXED = 1

EXPORTS = ["pcg_default_opts", "fem_assemble", "fem_dofs", "fem_csr", "fem_rhs", "fem_spmv", "fem_spmv_noalloc",
           "pcg_solve",
           "pcg_solve_batch", "pcg_stats", "fem_tune", "pcg_tune", "fem_set_format", "fem_set_tiling", "pcg_time_kernel", "pcg_time_spmm_cold", "bicgstab_solve",
           "fem_free",
           "fem_last_error", "serve_create", "serve_submit", "serve_step", "serve_poll", "serve_clock",
           "serve_destroy", "chol_analyze", "chol_factor", "chol_solve", "chol_stats", "chol_free"]


class FemcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("femcg error %d: %s" % (code, msg))
        self.code = code


class fem_mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nverts", C.c_int64), ("coords", C.c_void_p), ("ncells", C.c_int64),
                ("cells", C.c_void_p), ("on_boundary", C.c_void_p)]


class pcg_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("precision", C.c_int32),
                ("inner_eta", C.c_double), ("check_every", C.c_int32), ("use_x0", C.c_int32),
                ("max_restarts", C.c_int32), ("max_outer", C.c_int32), ("use_graph", C.c_int32)]


class chol_stats_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz_l", C.c_int64), ("nodes", C.c_int32), ("levels", C.c_int32),
                ("max_front", C.c_int32), ("pad", C.c_int32), ("flops", C.c_double), ("factor_mb", C.c_double),
                ("work_mb", C.c_double), ("order_s", C.c_double), ("symbolic_s", C.c_double),
                ("factor_s", C.c_double), ("total_s", C.c_double), ("solve_s", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad"}


class pcg_tune_report(C.Structure):
    _fields_ = [("format", C.c_int32), ("C", C.c_int32), ("sigma", C.c_int32), ("sfc", C.c_int32),
                ("lpr", C.c_int32), ("band", C.c_int32), ("tile", C.c_int32), ("ntiles", C.c_int32),
                ("precision", C.c_int32), ("fp64_fallback", C.c_int32), ("inner_eta", C.c_double),
                ("fp64_ms", C.c_double), ("mixed_ms", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class pcg_stats_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("nnz_nonzero", C.c_int64), ("nnz_stored", C.c_int64),
                ("k", C.c_int32), ("status", C.c_int32), ("precision", C.c_int32), ("format", C.c_int32),
                ("outer", C.c_int32), ("graph_replays", C.c_int32), ("iters", C.c_int64 * FEMCG_MAX_K),
                ("relres", C.c_double * FEMCG_MAX_K), ("setup_s", C.c_double), ("solve_s", C.c_double),
                ("bytes", C.c_double), ("gbps", C.c_double), ("gflops", C.c_double),
                ("footprint_mb", C.c_double)]

    def as_dict(self):
        k = self.k
        return dict(n=self.n, nnz=self.nnz, nnz_nonzero=self.nnz_nonzero, nnz_stored=self.nnz_stored, k=k,
                    status=self.status, precision=self.precision, format=self.format, outer=self.outer,
                    graph_replays=self.graph_replays, iters=[int(v) for v in self.iters[:k]],
                    relres=[float(v) for v in self.relres[:k]], setup_s=self.setup_s, solve_s=self.solve_s,
                    bytes=self.bytes, gbps=self.gbps, gflops=self.gflops, footprint_mb=self.footprint_mb)


class bicgstab_stats_t(C.Structure):
    _fields_ = [("iters", C.c_int64), ("relres", C.c_double), ("restarts", C.c_int32), ("block_size", C.c_int32),
                ("nblocks", C.c_int64), ("setup_s", C.c_double), ("solve_s", C.c_double), ("bytes", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class fem_request_info(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int32), ("k", C.c_int32), ("n", C.c_int64),
                ("iters_max", C.c_int64), ("t_submit", C.c_double), ("t_ready", C.c_double),
                ("t_admit", C.c_double),
                ("t_done", C.c_double), ("relres_max", C.c_double), ("footprint_mb", C.c_double)]


_lib = None


def lib():
    """Load libfemcg.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FemcgError(FEMCG_EDEVICE, "libfemcg.so is not built (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "pcg_default_opts": (None, [C.POINTER(pcg_opts)]),
        "fem_assemble": (C.c_int, [C.POINTER(fem_mesh), I32, I32, C.POINTER(P)]),
        "fem_dofs": (C.c_int, [P, C.POINTER(I64), C.POINTER(I64), P, P, P]),
        "fem_csr": (C.c_int, [P, C.POINTER(I64), P, P, P]),
        "fem_rhs": (C.c_int, [P, P, I32, P, P]),
        "fem_spmv": (C.c_int, [P, P, P, I32, P]),
        "fem_spmv_noalloc": (C.c_int, [P, P, P, I32, P]),
        "pcg_solve": (C.c_int, [P, P, P, I32, D, C.POINTER(pcg_opts), P]),
        "pcg_solve_batch": (C.c_int, [I32, P, P, P, P, P, C.POINTER(pcg_opts), P, P]),
        "pcg_stats": (C.c_int, [P, C.POINTER(pcg_stats_t)]),
        "fem_tune": (C.c_int, [P, I32, I32, C.POINTER(I32), C.POINTER(I32), P]),
        "pcg_tune": (C.c_int, [P, P, I32, D, C.POINTER(pcg_opts), C.POINTER(pcg_tune_report), P]),
        "chol_analyze": (C.c_int, [P, C.POINTER(chol_stats_t), P]),
        "chol_factor": (C.c_int, [P, C.POINTER(P), P]),
        "chol_solve": (C.c_int, [P, P, P, I32, P]),
        "chol_stats": (C.c_int, [P, C.POINTER(chol_stats_t)]),
        "chol_free": (None, [P]),
        "fem_set_format": (C.c_int, [P, I32, I32, I32]),
        "fem_set_tiling": (C.c_int, [P, I32, I32]),
        "pcg_time_kernel": (C.c_int, [P, I32, I32, P, C.POINTER(D), C.POINTER(D)]),
        "pcg_time_spmm_cold": (C.c_int, [I32, P, I32, I32, I32, P, C.POINTER(D), C.POINTER(D)]),
        "bicgstab_solve": (C.c_int, [P, P, P, D, I32, P, I64, P, C.POINTER(bicgstab_stats_t)]),
        "fem_free": (None, [P]),
        "fem_last_error": (C.c_char_p, []),
        "serve_create": (C.c_int, [D, I32, I32, I32, C.POINTER(P)]),
        "serve_submit": (I64, [P, C.POINTER(fem_mesh), I32, P, I32, D]),
        "serve_step": (C.c_int, [P]),
        "serve_poll": (C.c_int, [P, I64, P, C.POINTER(fem_request_info)]),
        "serve_clock": (D, [P]),
        "serve_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc):
    if rc < 0:
        raise FemcgError(rc, lib().fem_last_error().decode())
    return rc


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t, dtype_name="float64"):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous() or str(t.dtype) != "torch." + dtype_name:
        raise TypeError("expected a contiguous %s tensor" % dtype_name)
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def make_mesh_struct(mesh):
    coords = np.ascontiguousarray(mesh["coords"], dtype=np.float64)
    cells = np.ascontiguousarray(mesh["cells"], dtype=np.int32)
    bnd = np.ascontiguousarray(mesh["on_boundary"], dtype=np.uint8)
    m = fem_mesh(int(coords.shape[1]), coords.shape[0], _np_ptr(coords), cells.shape[0], _np_ptr(cells),
                 _np_ptr(bnd))
    return m, (coords, cells, bnd)


def default_opts(**kw):
    o = pcg_opts()
    lib().pcg_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Matrix:
    """An assembled system (fem_matrix*)."""

    def __init__(self, mesh, order, fmt=FEM_FORMAT_SELL):
        m, keep = make_mesh_struct(mesh)
        h = C.c_void_p()
        _check(lib().fem_assemble(C.byref(m), order, fmt, C.byref(h)))
        self.h = h
        self.dim = int(keep[0].shape[1])
        n_all, n_free = C.c_int64(), C.c_int64()
        _check(lib().fem_dofs(h, C.byref(n_all), C.byref(n_free), None, None, None))
        self.n_all, self.n_free = n_all.value, n_free.value

    def free(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.fem_free(h)
        self.h = None

    def __del__(self):
        self.free()

    def dofs(self):
        coords = np.zeros((self.n_all, self.dim))
        dirich = np.zeros(self.n_all, dtype=np.uint8)
        f2d = np.zeros(self.n_free, dtype=np.int64)
        _check(lib().fem_dofs(self.h, None, None, _np_ptr(coords), _np_ptr(dirich), _np_ptr(f2d)))
        return coords, dirich, f2d

    def csr(self):
        nnz = C.c_int64()
        _check(lib().fem_csr(self.h, C.byref(nnz), None, None, None))
        rp = np.zeros(self.n_free + 1, dtype=np.int64)
        col = np.zeros(max(nnz.value, 1), dtype=np.int32)
        val = np.zeros(max(nnz.value, 1))
        _check(lib().fem_csr(self.h, None, _np_ptr(rp), _np_ptr(col), _np_ptr(val)))
        return rp, col[: nnz.value], val[: nnz.value]

    def stats(self):
        s = pcg_stats_t()
        _check(lib().pcg_stats(self.h, C.byref(s)))
        return s.as_dict()


def fem_assemble(mesh, order, fmt=FEM_FORMAT_SELL):
    return Matrix(mesh, order, fmt)


def fem_rhs(A, g_all, B, stream=None):
    g = np.ascontiguousarray(g_all, dtype=np.float64)
    if g.ndim == 1:
        g = g[:, None]
    k = g.shape[1]
    if B.shape != (A.n_free, k):
        raise ValueError("B must be [n_free][k]")
    _check(lib().fem_rhs(A.h, _np_ptr(g), k, _dev_ptr(B), _stream(stream)))
    return B


def fem_spmv(A, X, Y, stream=None):
    k = X.shape[1]
    _check(lib().fem_spmv(A.h, _dev_ptr(X), _dev_ptr(Y), k, _stream(stream)))
    return Y


def fem_spmv_noalloc(A, X, Y, stream=None):
    """fem_spmv without allocation (the library's fixed scratch array);
    asynchronous on the stream."""
    k = X.shape[1]
    if X.shape != (A.n_free, k) or Y.shape != X.shape:
        raise ValueError("X and Y must be [n_free][k]")
    _check(lib().fem_spmv_noalloc(A.h, _dev_ptr(X), _dev_ptr(Y), k, _stream(stream)))
    return Y


FEMCG_NOALLOC_SCRATCH_BYTES = 64 << 20


def pcg_solve(A, B, X, tol, opts=None, stream=None):
    k = B.shape[1]
    if X.shape != B.shape or B.shape[0] != A.n_free:
        raise ValueError("B and X must be [n_free][k]")
    o = opts if opts is not None else default_opts(tol=tol)
    o.tol = tol
    return _check(lib().pcg_solve(A.h, _dev_ptr(B), _dev_ptr(X), k, tol, C.byref(o), _stream(stream)))


def bicgstab_solve(A, B, X, tol, block_size=1, max_iter=0, stream=None, row_scale=None):
    """BiCGStab + Block-Jacobi (exact blocks of block_size rows); B, X device
    [n_free] or [n_free][1] FP64; row_scale: None or host [n_free] positive
    values D (solves D A x = D b).  Returns (status, stats dict)."""
    if B.numel() != A.n_free or X.numel() != A.n_free:
        raise ValueError("B and X must hold n_free values (one right-hand side)")
    d = None
    if row_scale is not None:
        d = np.ascontiguousarray(row_scale, dtype=np.float64).reshape(-1)
        if d.size != A.n_free:
            raise ValueError("row_scale must hold n_free values")
    st = bicgstab_stats_t()
    rc = _check(lib().bicgstab_solve(A.h, _dev_ptr(B), _dev_ptr(X), tol, block_size,
                                     None if d is None else _np_ptr(d), max_iter, _stream(stream), C.byref(st)))
    return rc, st.as_dict()


def pcg_solve_batch(As, Bs, Xs, tols, opts=None, stream=None):
    n = len(As)
    hs = (C.c_void_p * n)(*[a.h for a in As])
    bp = (C.c_void_p * n)(*[_dev_ptr(b).value for b in Bs])
    xp = (C.c_void_p * n)(*[_dev_ptr(x).value for x in Xs])
    ks = (C.c_int32 * n)(*[b.shape[1] for b in Bs])
    ts = (C.c_double * n)(*tols)
    st = (C.c_int32 * n)()
    o = opts if opts is not None else default_opts()
    _check(lib().pcg_solve_batch(n, hs, bp, xp, ks, ts, C.byref(o), st, _stream(stream)))
    return list(st)


def pcg_stats(A):
    return A.stats()


def fem_set_format(A, fmt, Cw=64, sigma=1):
    return _check(lib().fem_set_format(A.h, fmt, Cw, sigma))


def fem_set_tiling(A, band=-1, tile=0):
    return _check(lib().fem_set_tiling(A.h, band, tile))


def fem_tune(A, k, precision=PCG_FP64, stream=None):
    cw, sg = C.c_int32(), C.c_int32()
    f = _check(lib().fem_tune(A.h, k, precision, C.byref(cw), C.byref(sg), _stream(stream)))
    return f, cw.value, sg.value


def pcg_tune(A, B, tol, opts=None, stream=None):
    """Autotune format, lanes per row, tiling, precision and inner_eta on the
    solve of B to tol; returns (tuned pcg_opts, report dict)."""
    k = B.shape[1]
    if B.shape[0] != A.n_free:
        raise ValueError("B must be [n_free][k]")
    o = opts if opts is not None else default_opts(tol=tol)
    rep = pcg_tune_report()
    _check(lib().pcg_tune(A.h, _dev_ptr(B), k, tol, C.byref(o), C.byref(rep), _stream(stream)))
    return o, rep.as_dict()


def chol_analyze(A):
    """Nested-dissection ordering and symbolic analysis of A (host only):
    returns (stats dict, perm), perm[p] = free row at elimination position p."""
    import numpy as np
    st = chol_stats_t()
    perm = np.zeros(max(A.n_free, 1), dtype=np.int32)
    _check(lib().chol_analyze(A.h, C.byref(st), _np_ptr(perm)))
    return st.as_dict(), perm[: A.n_free]


class Chol:
    """Sparse Cholesky factor of A = K_II on the device (chol_factor)."""

    def __init__(self, A, stream=None):
        self.h = C.c_void_p()
        self.n = A.n_free
        _check(lib().chol_factor(A.h, C.byref(self.h), _stream(stream)))

    def solve(self, B, X, stream=None):
        if B.shape != X.shape or B.shape[0] != self.n:
            raise ValueError("B and X must be [n_free][k]")
        _check(lib().chol_solve(self.h, _dev_ptr(B), _dev_ptr(X), B.shape[1], _stream(stream)))
        return X

    def stats(self):
        st = chol_stats_t()
        _check(lib().chol_stats(self.h, C.byref(st)))
        return st.as_dict()

    def free(self):
        if self.h:
            lib().chol_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def pcg_time_spmm_cold(mats, k, precision=PCG_FP64, reps=5, stream=None):
    arr = (C.c_void_p * len(mats))(*[m.h for m in mats])
    ms, by = C.c_double(), C.c_double()
    _check(lib().pcg_time_spmm_cold(len(mats), arr, k, precision, reps, _stream(stream), C.byref(ms),
                                    C.byref(by)))
    return ms.value, by.value


def pcg_time_kernel(A, kernel, reps=20, stream=None):
    ms, by = C.c_double(), C.c_double()
    _check(lib().pcg_time_kernel(A.h, kernel, reps, _stream(stream), C.byref(ms), C.byref(by)))
    return ms.value, by.value
