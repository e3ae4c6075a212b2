"""Pins of the oracle's checkers: the product A X of the MatMult step
(Sect. 3.2) for k interleaved columns, the relative residual of Eq. (2) and
the error of Eq. (1).  Every GPU residual gate and every SpMM parity test
trusts these three, so each is fixed here by a closed form that does not come
from the oracle itself:

* on the structured 2D grid the lifted P1 matrix is the 5-point stencil
  (4, -1) on the interior nodes, whose eigenvectors are the discrete sines
  sin(p pi x) sin(q pi y) with eigenvalue 4 sin^2(p pi h/2) + 4 sin^2(q pi h/2);
  on the structured Kuhn cube it is h times the 7-point stencil (6, -1), with
  the analogous three-term eigenvalues.  Each column carries its own mode, so
  a product that mixes, transposes or drops columns fails;
* the product also equals scipy's CSR product of the exported matrix on a
  jittered P2 mesh (a second summation, no shared code);
* Eq. (2): relres(B, 0) = 1 exactly in every column; relres(B, X*) sits at
  rounding level when X* is the exact discrete solution (linear data on P1,
  the patch test); moving one entry (i, j) of X* by delta gives
  delta ||A e_i|| / ||b_j|| in column j alone, with ||A e_i|| = sqrt(20) for
  an interior node whose four neighbours are free and sqrt(19) when one of
  them is a Dirichlet node (5-point stencil);
* Eq. (1): the norm of the difference over the norm of the first argument.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle


def _five_point_system(m):
    s = oracle.System(meshgen.mesh2d(m), 1)
    coords, _, f2d = s.dofs()
    return s, coords[f2d], 1.0 / (m - 1)


def test_spmv_sine_eigenvectors_2d_columns_distinct():
    s, xy, h = _five_point_system(23)
    modes = [(1, 1), (2, 5), (7, 3), (4, 4), (11, 2)]
    k = len(modes)
    U = np.stack([np.sin(p * math.pi * xy[:, 0]) * np.sin(q * math.pi * xy[:, 1]) for p, q in modes], 1)
    lam = np.array([4 * math.sin(p * math.pi * h / 2) ** 2 + 4 * math.sin(q * math.pi * h / 2) ** 2
                    for p, q in modes])
    Y = s.spmv(U)
    assert Y.shape == (s.nfree, k)
    for j in range(k):
        assert np.max(np.abs(Y[:, j] - lam[j] * U[:, j])) <= 1e-13, j
    # the modes are distinct, so a column mix-up cannot pass by accident
    assert np.min(np.abs(np.diff(np.sort(lam)))) > 1e-2


def test_spmv_sine_eigenvectors_3d_kuhn():
    m = 10
    s = oracle.System(meshgen.mesh3d(m), 1)
    coords, _, f2d = s.dofs()
    x = coords[f2d]
    h = 1.0 / (m - 1)
    modes = [(1, 1, 1), (2, 3, 1), (5, 1, 4)]
    U = np.stack([np.sin(a * math.pi * x[:, 0]) * np.sin(b * math.pi * x[:, 1]) *
                  np.sin(c * math.pi * x[:, 2]) for a, b, c in modes], 1)
    Y = s.spmv(U)
    for j, (a, b, c) in enumerate(modes):
        lam = h * sum(4 * math.sin(t * math.pi * h / 2) ** 2 for t in (a, b, c))
        # the Kuhn stiffness also holds exact zeros that cancel to rounding level
        assert np.max(np.abs(Y[:, j] - lam * U[:, j])) <= 1e-14, j


def test_spmv_equals_scipy_csr_product_jittered_p2():
    s = oracle.System(meshgen.mesh2d(13, 0.25, 7), 2)
    rp, col, val = s.A()
    A = sp.csr_matrix((val, col, rp), shape=(s.nfree, s.nfree))
    X = meshgen.noise(21, s.nfree * 6, 1.0).reshape(s.nfree, 6)
    Y = s.spmv(X)
    Yr = A @ X
    scale = np.abs(A).max() * np.abs(X).max()
    assert np.max(np.abs(Y - Yr)) <= 1e-13 * scale
    # one column at a time gives the same bits as the interleaved call
    for j in range(6):
        assert np.array_equal(s.spmv(np.ascontiguousarray(X[:, j]))[:, 0], Y[:, j])


def _linear_columns(coords, f2d):
    lin = [(1.0, 2.0, -3.0), (-0.5, 0.25, 4.0), (2.0, -1.0, 0.5)]
    g = np.stack([a + b * coords[:, 0] + c * coords[:, 1] for a, b, c in lin], 1)
    return g, g[f2d]


def test_relres_zero_guess_is_one_every_column():
    s = oracle.System(meshgen.mesh2d(17, 0.3, 3), 1)
    coords, _, f2d = s.dofs()
    g, _ = _linear_columns(coords, f2d)
    B = s.rhs(g)
    B[:, 1] *= 1e3  # columns of very different size
    rel = s.relres(B, np.zeros_like(B))
    assert rel.shape == (3,)
    assert np.array_equal(rel, np.ones(3))


def test_relres_exact_solution_at_rounding_level_jittered():
    s = oracle.System(meshgen.mesh2d(17, 0.3, 3), 1)
    coords, _, f2d = s.dofs()
    g, Xs = _linear_columns(coords, f2d)
    B = s.rhs(g)
    rel = s.relres(B, Xs)
    assert np.all(rel <= 1e-14), rel
    # b = 0 and x = 0 gives 0 (the stated convention), beside a live column
    B2 = np.concatenate([B[:, :1], np.zeros((s.nfree, 1))], 1)
    X2 = np.concatenate([Xs[:, :1], np.zeros((s.nfree, 1))], 1)
    rel2 = s.relres(B2, X2)
    assert rel2[1] == 0.0 and rel2[0] <= 1e-14


def test_relres_single_entry_perturbation_closed_form():
    m = 15
    s, xy, h = _five_point_system(m)
    coords, _, f2d = s.dofs()
    g, Xs = _linear_columns(coords, f2d)
    B = s.rhs(g)
    nb = np.linalg.norm(B, axis=0)
    n_in = m - 2  # interior nodes per side; free DOF (a, b) -> index a * n_in + b or b * n_in + a

    def free_index(ix, iy):
        # locate the free DOF at grid node (ix, iy) from its coordinates
        d = np.abs(xy[:, 0] - ix * h) + np.abs(xy[:, 1] - iy * h)
        i = int(np.argmin(d))
        assert d[i] < 1e-12
        return i

    cases = [(0, free_index(5, 6), math.sqrt(20.0)),    # four free neighbours
             (1, free_index(1, 7), math.sqrt(19.0)),    # one neighbour on the boundary
             (2, free_index(n_in, n_in), math.sqrt(18.0))]  # corner: two on the boundary
    for j, i, col_norm in cases:
        delta = 1e-5 * nb[j]
        X = Xs.copy()
        X[i, j] += delta
        rel = s.relres(B, X)
        expect = delta * col_norm / nb[j]
        assert abs(rel[j] - expect) <= 1e-6 * expect, (j, rel[j], expect)
        for jj in range(3):
            if jj != j:
                assert rel[jj] <= 1e-14, (j, jj, rel[jj])


def test_x_err_definition():
    assert oracle.x_err(np.array([3.0, 4.0]), np.array([3.0, 4.0])) == 0.0
    # denominator is the first argument's norm
    assert oracle.x_err(np.array([6.0, 8.0]), np.array([3.0, 4.0])) == pytest.approx(0.5, rel=1e-15)
    assert oracle.x_err(np.array([3.0, 4.0]), np.array([6.0, 8.0])) == pytest.approx(1.0, rel=1e-15)
    # 2D arrays: one norm over all entries
    a = np.array([[3.0, 0.0], [0.0, 4.0]])
    b = np.array([[3.0, 0.0], [0.0, 4.0 + 5e-3]])
    assert oracle.x_err(a, b) == pytest.approx(1e-3, rel=1e-12)
