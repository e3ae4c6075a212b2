"""Plain CPU FP64 oracle for the FEM Laplace / Jacobi-PCG path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark load this package; the library never does.  It
shares no code with the HIP library.  The arithmetic lives in
``femoracle.c`` (plain C, FP64); this module only marshals numpy arrays.

Each wrapper names the passage of the paper the C function follows:

* ``p1_element`` / ``p1_element_cot`` -- the Laplacian weights of Sect. 2.2
  (gradient form and the paper's cotangent form, K_ij = -w(i,j));
* ``p2_element`` -- Table 7's higher-degree basis (degree 2), exact quadrature;
* ``pk_element`` -- Table 7's degrees 3 and 4 on triangles: nodal basis from
  the inverse Vandermonde matrix, collapsed Gauss-Legendre quadrature;
* ``bicgstab_csr`` / ``bj_apply`` -- the paper's own iterative solver
  (Sect. 3.2): BiCGStab right preconditioned by Block-Jacobi with exact
  blocks of bs consecutive rows;
* ``System`` -- assembly, Dirichlet lifting (Sect. 2.2: u = f on the boundary,
  b encodes the boundary condition), Jacobi-PCG (Sect. 2.1, M = diag(A)) with
  the exit test of Eq. (2), and the error metric of Eq. (1).

Pins (tests/test_oracle_*.py) tie every function to something other than
itself: closed-form stencils, patch tests, dense LU, the paper's Table 1 counts.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "femoracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_omp = None

ERRORS = {-1: "invalid argument", -2: "out of memory", -3: "invalid mesh (non-positive cell)",
          -4: "breakdown (p.Ap <= 0)"}


def build(force: bool = True) -> str:
    """Compile femoracle.c with gcc into liboracle.so (plain -O2, one thread),
    and the same source with -fopenmp into liboracle_omp.so, the all-core
    timing build of the CPU baseline (independent columns on separate
    threads; per-column arithmetic unchanged)."""
    for path, extra in ((_LIB_PATH, []), (_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared"] + extra + ["-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB_PATH


def _load(omp: bool = False):
    global _lib, _omp
    if (_omp if omp else _lib) is not None:
        return _omp if omp else _lib
    path = _OMP_PATH if omp else _LIB_PATH
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.orc_p1_element.argtypes = [C.c_int, P, P]
    lib.orc_p1_element_cot.argtypes = [C.c_int, P, P]
    lib.orc_p2_element.argtypes = [C.c_int, P, P]
    lib.orc_pk_element.argtypes = [C.c_int, P, P]
    lib.orc_build.argtypes = [C.c_int, C.c_int64, P, C.c_int64, P, P, C.c_int, C.POINTER(C.c_int)]
    lib.orc_build.restype = P
    lib.orc_free.argtypes = [P]
    lib.orc_sizes.argtypes = [P, P]
    lib.orc_copy_dofs.argtypes = [P, P, P, P]
    lib.orc_copy_K.argtypes = [P, P, P, P]
    lib.orc_copy_A.argtypes = [P, P, P, P]
    lib.orc_rhs.argtypes = [P, P, C.c_int, P]
    lib.orc_spmv.argtypes = [P, P, C.c_int, P]
    lib.orc_relres.argtypes = [P, P, P, C.c_int, P]
    lib.orc_pcg.argtypes = [P, P, C.c_int, C.c_double, C.c_int64, P, P, P, P]
    lib.orc_pcg_csr.argtypes = [C.c_int64, P, P, P, P, C.c_int, C.c_double, C.c_int64, P, P, P, P]
    lib.orc_bj_apply.argtypes = [C.c_int64, P, P, P, C.c_int, P, P]
    lib.orc_bicgstab_csr.argtypes = [C.c_int64, P, P, P, P, C.c_int, C.c_double, C.c_int64, P, P, P, P]
    lib.orc_fd7_identity_nnz.argtypes = [C.c_int64]
    lib.orc_fd7_identity_nnz.restype = C.c_int64
    lib.orc_threads.argtypes = [C.c_int]
    lib.orc_dense_cholesky.argtypes = [C.c_int64, P, P, P, P, C.c_int, P, P]
    if omp:
        _omp = lib
    else:
        _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _check(rc):
    if rc < 0:
        raise RuntimeError("oracle error %d: %s" % (rc, ERRORS.get(rc, "?")))
    return rc


def _element(fn, dim, X, nloc):
    X = np.ascontiguousarray(X, dtype=np.float64)
    K = np.zeros((nloc, nloc))
    _check(fn(dim, _ptr(X), _ptr(K)))
    return K


def p1_element(X: np.ndarray) -> np.ndarray:
    """P1 element stiffness, gradient form, for a simplex X[(d+1)][d]."""
    dim = X.shape[1]
    return _element(_load().orc_p1_element, dim, X, dim + 1)


def p1_element_cot(X: np.ndarray) -> np.ndarray:
    """P1 element stiffness from the cotangent weights of Sect. 2.2."""
    dim = X.shape[1]
    return _element(_load().orc_p1_element_cot, dim, X, dim + 1)


def p2_element(X: np.ndarray) -> np.ndarray:
    """P2 element stiffness; local order: vertices, then edges (a,b), a<b, lexicographic."""
    dim = X.shape[1]
    return _element(_load().orc_p2_element, dim, X, 6 if dim == 2 else 10)


def pk_element(X: np.ndarray, k: int) -> np.ndarray:
    """P3/P4 triangle stiffness (Table 7's degrees 3 and 4); local order:
    lattice points (i/k, j/k) of the reference triangle, i outer, j inner."""
    return _element(lambda d, x, K: _load().orc_pk_element(k, x, K), 2, X, (k + 1) * (k + 2) // 2)


def pk_local_points(k: int) -> np.ndarray:
    """Barycentric indices (k-i-j, i, j) of the local numbering of pk_element."""
    return np.array([(k - i - j, i, j) for i in range(k + 1) for j in range(k - i + 1)], dtype=np.int64)


def fd7_identity_nnz(m: int) -> int:
    """Nonzeros of the 7-point FD matrix on m^3 nodes with identity Dirichlet rows."""
    return int(_load().orc_fd7_identity_nnz(m))


class System:
    """Assembled FEM system of one mesh: full stiffness K, lifted A = K_II."""

    def __init__(self, mesh, order: int):
        lib = _load()
        coords = np.ascontiguousarray(mesh["coords"], dtype=np.float64)
        cells = np.ascontiguousarray(mesh["cells"], dtype=np.int32)
        bnd = np.ascontiguousarray(mesh["on_boundary"], dtype=np.uint8)
        self.dim = int(coords.shape[1])
        self.order = order
        err = C.c_int(0)
        h = lib.orc_build(self.dim, coords.shape[0], _ptr(coords), cells.shape[0], _ptr(cells),
                          _ptr(bnd), order, C.byref(err))
        if not h:
            _check(err.value)
            raise RuntimeError("oracle build failed")
        self._h = h
        sz = np.zeros(6, dtype=np.int64)
        lib.orc_sizes(h, _ptr(sz))
        self.ndofs, self.nedges, self.nfree, self.nnz_K, self.nnz_A, self.nloc = (int(v) for v in sz)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    # -- accessors --
    def dofs(self):
        coords = np.zeros((self.ndofs, self.dim))
        dirich = np.zeros(self.ndofs, dtype=np.uint8)
        free2dof = np.zeros(self.nfree, dtype=np.int64)
        _load().orc_copy_dofs(self._h, _ptr(coords), _ptr(dirich), _ptr(free2dof))
        return coords, dirich, free2dof

    def K(self):
        rp = np.zeros(self.ndofs + 1, dtype=np.int64)
        col = np.zeros(max(self.nnz_K, 1), dtype=np.int32)
        val = np.zeros(max(self.nnz_K, 1))
        _load().orc_copy_K(self._h, _ptr(rp), _ptr(col), _ptr(val))
        return rp, col[: self.nnz_K], val[: self.nnz_K]

    def A(self):
        rp = np.zeros(self.nfree + 1, dtype=np.int64)
        col = np.zeros(max(self.nnz_A, 1), dtype=np.int32)
        val = np.zeros(max(self.nnz_A, 1))
        _load().orc_copy_A(self._h, _ptr(rp), _ptr(col), _ptr(val))
        return rp, col[: self.nnz_A], val[: self.nnz_A]

    # -- the path --
    def rhs(self, g_all: np.ndarray) -> np.ndarray:
        """b = -K_ID g_D, g_all [ndofs][k] -> B [nfree][k]."""
        g = np.ascontiguousarray(g_all, dtype=np.float64)
        if g.ndim == 1:
            g = g[:, None]
        k = g.shape[1]
        B = np.zeros((self.nfree, k))
        _check(_load().orc_rhs(self._h, _ptr(g), k, _ptr(B)))
        return B

    def spmv(self, X: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float64)
        if X.ndim == 1:
            X = X[:, None]
        Y = np.zeros_like(X)
        _check(_load().orc_spmv(self._h, _ptr(X), X.shape[1], _ptr(Y)))
        return Y

    def relres(self, B: np.ndarray, X: np.ndarray) -> np.ndarray:
        """Eq. (2) per column: ||b - A x|| / ||b||."""
        B = np.ascontiguousarray(B, dtype=np.float64).reshape(self.nfree, -1)
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(self.nfree, -1)
        k = B.shape[1]
        out = np.zeros(k)
        _check(_load().orc_relres(self._h, _ptr(B), _ptr(X), k, _ptr(out)))
        return out

    def pcg(self, B: np.ndarray, tol: float, max_iter: int | None = None):
        """Jacobi-PCG per column; returns X, iters, relres, restarts, status."""
        B = np.ascontiguousarray(B, dtype=np.float64)
        if B.ndim == 1:
            B = B[:, None]
        k = B.shape[1]
        if max_iter is None:
            max_iter = default_max_iter(self.nfree)
        X = np.zeros_like(B)
        its = np.zeros(k, dtype=np.int64)
        rel = np.zeros(k)
        rs = np.zeros(k, dtype=np.int32)
        st = _check(_load().orc_pcg(self._h, _ptr(B), k, tol, max_iter, _ptr(X), _ptr(its),
                                    _ptr(rel), _ptr(rs)))
        return X, its, rel, rs, st

    def scatter(self, X_free: np.ndarray, g_all: np.ndarray) -> np.ndarray:
        """Full nodal vector: x on free DOFs, g on Dirichlet DOFs."""
        _, dirich, free2dof = self.dofs()
        g = np.array(g_all, dtype=np.float64).reshape(self.ndofs, -1)
        u = g.copy()
        u[free2dof] = np.asarray(X_free).reshape(self.nfree, -1)
        return u


def pcg_csr(rowptr, col, val, B, tol, max_iter=None, threads=0):
    """The oracle's Jacobi-PCG on a caller-given CSR matrix (planted-defect
    tests).  threads > 0 runs the all-core build (the CPU baseline's timing
    build): the k columns on that many threads, each with the same
    arithmetic, so the results are identical.  Returns X, iterations,
    relres, restarts, status."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    n, k = B.shape
    if max_iter is None:
        max_iter = default_max_iter(n)
    X = np.zeros_like(B)
    its = np.zeros(k, dtype=np.int64)
    rel = np.zeros(k)
    rs = np.zeros(k, dtype=np.int32)
    lib = _load(omp=threads > 0)
    if threads > 0:
        lib.orc_threads(threads)
    st = lib.orc_pcg_csr(n, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(B), k, tol, max_iter,
                         _ptr(X), _ptr(its), _ptr(rel), _ptr(rs))
    return X, its, rel, rs, st


def omp_threads() -> int:
    """Threads the all-core build runs on (OMP_NUM_THREADS or all host cores)."""
    return int(_load(omp=True).orc_threads(0))


def bj_apply(rowptr, col, val, bs, r):
    """z = M^-1 r for the Block-Jacobi preconditioner with exact blocks of bs
    consecutive rows (Sect. 3.2's preconditioner)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    _check(_load().orc_bj_apply(len(rowptr) - 1, _ptr(rowptr), _ptr(col), _ptr(val), bs, _ptr(r), _ptr(z)))
    return z


def bicgstab_csr(rowptr, col, val, b, bs, tol, max_iter=None):
    """BiCGStab, right preconditioned by Block-Jacobi (exact blocks of bs
    consecutive rows), zero initial guess (Sect. 3.2's solver).  Returns
    x, iterations, true relative residual, restarts, status."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
    n = len(rowptr) - 1
    if max_iter is None:
        max_iter = default_max_iter(n)
    x = np.zeros(n)
    its = np.zeros(1, dtype=np.int64)
    rel = np.zeros(1)
    rs = np.zeros(1, dtype=np.int32)
    st = _load().orc_bicgstab_csr(n, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(b), bs, tol, max_iter, _ptr(x),
                                  _ptr(its), _ptr(rel), _ptr(rs))
    return x, int(its[0]), float(rel[0]), int(rs[0]), st


def dense_cholesky(rowptr, col, val, B=None, want_L=False):
    """Direct solve of the SPD system by dense Cholesky (Sect. 4.3's direct
    solver: factorise once, forward and backward substitution per
    right-hand side).  Returns (X or None, L or None, status)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    n = len(rowptr) - 1
    X = Bc = None
    k = 0
    if B is not None:
        Bc = np.ascontiguousarray(B, dtype=np.float64).reshape(n, -1)
        k = Bc.shape[1]
        X = np.zeros_like(Bc)
    L = np.zeros((n, n)) if want_L else None
    st = _load().orc_dense_cholesky(n, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(Bc) if Bc is not None else None, k,
                                    _ptr(X) if X is not None else None, _ptr(L) if L is not None else None)
    return X, L, st


def default_max_iter(n: int) -> int:
    """A generous cap: 20 sqrt(n) log2(n) + 100."""
    import math
    n = max(int(n), 2)
    return int(20 * math.sqrt(n) * math.log2(n) + 100)


def x_err(x_gt: np.ndarray, x: np.ndarray) -> float:
    """Eq. (1): ||x_gt - x||_2 / ||x_gt||_2."""
    x_gt = np.asarray(x_gt, dtype=np.float64).ravel()
    x = np.asarray(x, dtype=np.float64).ravel()
    return float(np.linalg.norm(x_gt - x) / np.linalg.norm(x_gt))
