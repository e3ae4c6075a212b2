"""Pins of the oracle's BiCGStab + Block-Jacobi (Sect. 3.2's iterative solver).

* the preconditioner: z = M^-1 r equals a block-diagonal solve built here
  with numpy (dense blocks of bs consecutive rows, the last one ragged); at
  bs = 1 it is r / diag(A);
* a single block holding every row makes M = A: BiCGStab then stops after
  one iteration (alpha = 1, s = 0) at x = A^-1 b;
* the solution equals a sparse direct solve (scipy) on the SPD FEM matrix
  and on the paper's nonsymmetric form B^-1 L (rows scaled by the lumped
  vertex areas), for several block sizes;
* a Lanczos near-breakdown (lifted b lives next to the boundary) restarts
  the iteration and it still reaches the direct solution;
* b = 0 gives x = 0 in 0 iterations; a singular diagonal block is reported.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import meshgen
import oracle


def _system(m=24, order=1, jit=0.3, seed=3):
    s = oracle.System(meshgen.mesh2d(m, jit, seed), order)
    rp, col, val = s.A()
    coords, _, _ = s.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(2, 1, seed + 10), coords)
    return s, rp, col, val, s.rhs(g)[:, 0]


@pytest.mark.parametrize("bs", [1, 3, 8, 64])
def test_block_jacobi_apply_is_a_block_diagonal_solve(bs):
    s, rp, col, val, _ = _system(m=14, order=2)
    n = s.nfree
    assert n % bs != 0 or bs == 1  # a ragged last block for bs > 1
    A = sp.csr_matrix((val, col, rp), shape=(n, n)).toarray()
    r = np.random.default_rng(bs).standard_normal(n)
    ref = np.zeros(n)
    for b0 in range(0, n, bs):
        b1 = min(n, b0 + bs)
        ref[b0:b1] = np.linalg.solve(A[b0:b1, b0:b1], r[b0:b1])
    z = oracle.bj_apply(rp, col, val, bs, r)
    assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()
    if bs == 1:
        assert np.abs(z - r / np.diag(A)).max() <= 1e-15 * np.abs(z).max()


def test_one_block_is_the_exact_inverse_and_stops_after_one_iteration():
    s, rp, col, val, b = _system(m=7, order=1)
    n = s.nfree
    assert n <= 64
    x, its, rel, rs, st = oracle.bicgstab_csr(rp, col, val, b, 64, 1e-12)
    A = sp.csr_matrix((val, col, rp), shape=(n, n)).toarray()
    assert st == 0 and its == 1 and rs == 0
    xs = np.linalg.solve(A, b)
    assert np.abs(x - xs).max() <= 1e-12 * np.abs(xs).max()


def _lumped_areas(mesh, s):
    """B of Sect. 2.2 for triangles: the area of the cells around each vertex."""
    X = np.asarray(mesh["coords"])
    T = np.asarray(mesh["cells"])
    a = 0.5 * np.abs((X[T[:, 1], 0] - X[T[:, 0], 0]) * (X[T[:, 2], 1] - X[T[:, 0], 1])
                     - (X[T[:, 2], 0] - X[T[:, 0], 0]) * (X[T[:, 1], 1] - X[T[:, 0], 1]))
    B = np.zeros(len(X))
    for j in range(3):
        np.add.at(B, T[:, j], a)
    _, _, f2d = s.dofs()
    return B[f2d]


@pytest.mark.parametrize("bs", [1, 4, 16])
@pytest.mark.parametrize("form", ["K", "BinvL"])
def test_solution_equals_sparse_direct_solve(bs, form):
    mesh = meshgen.mesh2d(26, 0.3, 4)
    s = oracle.System(mesh, 1)
    rp, col, val = s.A()
    coords, _, _ = s.dofs()
    b = s.rhs(meshgen.harmonic_eval(meshgen.random_coeffs(2, 1, 9), coords))[:, 0]
    if form == "BinvL":
        # the paper's A = B^-1 L (rows scaled): nonsymmetric, same solution
        d = 1.0 / _lumped_areas(mesh, s)
        val = val * np.repeat(d, np.diff(rp))
        b = b * d
    n = s.nfree
    A = sp.csr_matrix((val, col, rp), shape=(n, n))
    if form == "BinvL":
        assert abs(A - A.T).max() > 1e-3 * abs(A).max()
    xs = sla.spsolve(A.tocsc(), b)
    x, its, rel, rs, st = oracle.bicgstab_csr(rp, col, val, b, bs, 1e-12)
    assert st == 0 and rel <= 1e-12
    assert np.linalg.norm(A @ x - b) <= 1.0001e-12 * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_lanczos_near_breakdown_restarts_and_still_solves():
    # lifted Dirichlet data: b (the first shadow residual) lives on the rows
    # next to the boundary, and (rh, r) collapses long before r does
    s = oracle.System(meshgen.mesh2d(60, 0.3, 1), 1)
    coords, _, _ = s.dofs()
    b = s.rhs((coords[:, 0] ** 2 - coords[:, 1] ** 2)[:, None])[:, 0]
    assert np.count_nonzero(b) < 0.1 * len(b)
    rp, col, val = s.A()
    x, its, rel, rs, st = oracle.bicgstab_csr(rp, col, val, b, 4, 1e-10)
    assert st == 0 and rs >= 1 and rel <= 1e-10
    A = sp.csr_matrix((val, col, rp), shape=(s.nfree, s.nfree))
    xs = sla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)


def test_zero_rhs_and_singular_block():
    s, rp, col, val, b = _system(m=10)
    x, its, rel, rs, st = oracle.bicgstab_csr(rp, col, val, np.zeros_like(b), 4, 1e-10)
    assert st == 0 and its == 0 and not x.any()
    val2 = val.copy()
    val2[rp[0]:rp[1]] = 0.0  # first row empty: its 1x1 block is singular
    *_, st = oracle.bicgstab_csr(rp, col, val2, b, 1, 1e-10)
    assert st == -4  # breakdown


def test_unreachable_tol_warns_after_the_last_restart():
    # tol 1e-17 is below the rounding floor of the true residual: the
    # recursion converges, the true residual misses Eq. (2) three restarts in
    # a row, and the result is a warning (1), well before the iteration cap
    s, rp, col, val, b = _system(m=12)
    x, its, rel, rs, st = oracle.bicgstab_csr(rp, col, val, b, 4, 1e-17)
    assert st == 1 and rel > 1e-17 and rs == 3 and its < oracle.default_max_iter(s.nfree)
