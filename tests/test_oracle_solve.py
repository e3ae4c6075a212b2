"""Pins of the oracle's Jacobi-PCG (Sect. 2.1, M = diag(A); exit test Eq. (2)).

* tiny meshes: the PCG solution at tol 1e-14 equals a dense LU solve;
* the first configuration's data g = 1 + 2x - 3y is the exact discrete
  solution (Eq. (1) error at solver level);
* structured 3D Kuhn P1 reproduces harmonic cubics exactly (the stencil is
  h times the 7-point one, whose truncation error vanishes on cubics);
* iteration count on the 5-point matrix stays under the textbook CG bound
  0.5 sqrt(kappa) ln(2/tol) with kappa from the closed-form eigenvalues;
* degenerate input: b = 0 gives x = 0 in 0 iterations; an indefinite matrix
  reports breakdown; max_iter caps the count.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle


@pytest.mark.parametrize("dim,order,m,jit", [(2, 1, 14, 0.3), (2, 2, 9, 0.25), (3, 1, 8, 0.3),
                                             (3, 2, 5, 0.3)])
def test_pcg_equals_dense_lu(dim, order, m, jit):
    mesh = meshgen.make_mesh(dim, m, jit, 11)
    s = oracle.System(mesh, order)
    assert s.nfree <= 2000
    coords, _, _ = s.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(dim, 3, 12), coords)
    g += meshgen.noise(13, g.size, 0.01).reshape(g.shape)
    B = s.rhs(g)
    A = sp.csr_matrix((s.A()[2], s.A()[1], s.A()[0]), shape=(s.nfree, s.nfree)).toarray()
    Xd = np.linalg.solve(A, B)
    X, its, rel, rs, st = s.pcg(B, 1e-14)
    assert st == 0
    for j in range(3):
        assert oracle.x_err(Xd[:, j], X[:, j]) <= 1e-11
        assert rel[j] <= 1e-14
        r = B[:, j] - A @ X[:, j]
        assert abs(rel[j] - np.linalg.norm(r) / np.linalg.norm(B[:, j])) <= 1e-3 * rel[j] + 2e-15  # residual rounding floor


def test_c1_exact_linear_solution():
    w = meshgen.c1()
    s = oracle.System(w.mesh, 1)
    coords, _, f2d = s.dofs()
    g = w.dirichlet(coords)
    X, its, rel, rs, st = s.pcg(s.rhs(g), 1e-10)
    assert s.nfree == 62 * 62 == 3844
    assert st == 0 and rel[0] <= 1e-10
    assert oracle.x_err(g[f2d], X) <= 1e-9


def test_structured_3d_reproduces_harmonic_cubics():
    mesh = meshgen.mesh3d(12)
    s = oracle.System(mesh, 1)
    coords, _, f2d = s.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(3, 4, 3), coords)
    X, its, rel, rs, st = s.pcg(s.rhs(g), 1e-13)
    assert st == 0
    for j in range(4):
        assert oracle.x_err(g[f2d, j], X[:, j]) <= 1e-10


def test_iterations_within_cg_bound_on_5_point():
    m = 40
    s = oracle.System(meshgen.mesh2d(m), 1)
    coords, _, _ = s.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(2, 1, 1), coords)
    tol = 1e-10
    X, its, rel, rs, st = s.pcg(s.rhs(g), tol)
    n = m - 2
    lmin = 8 * math.sin(math.pi / (2 * (n + 1))) ** 2
    lmax = 8 * math.cos(math.pi / (2 * (n + 1))) ** 2
    kappa = lmax / lmin
    bound = 0.5 * math.sqrt(kappa) * math.log(2 / tol)
    assert its[0] <= bound
    assert its[0] >= 0.25 * math.sqrt(kappa)  # no miraculous shortcut either


def test_zero_rhs_and_max_iter_and_columns_independent():
    s = oracle.System(meshgen.mesh2d(20, 0.3, 1), 1)
    coords, _, _ = s.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(2, 2, 4), coords)
    B = s.rhs(g)
    B3 = np.concatenate([B[:, :1], np.zeros((s.nfree, 1)), B[:, 1:]], 1)
    X, its, rel, rs, st = s.pcg(B3, 1e-10)
    assert its[1] == 0 and np.all(X[:, 1] == 0.0) and rel[1] == 0.0
    X0, its0, _, _, _ = s.pcg(B[:, :1], 1e-10)
    assert np.array_equal(X0[:, 0], X[:, 0]) and its0[0] == its[0]
    Xc, itc, relc, _, stc = s.pcg(B[:, :1], 1e-10, max_iter=5)
    assert stc == 1 and itc[0] == 5 and relc[0] > 1e-10


def test_breakdown_reported():
    # plant a defect: negate the matrix (symmetric, negative definite); with
    # the Jacobi preconditioner p = D^-1 b the first p.Ap is negative, so the
    # recurrence must stop with the breakdown code
    s = oracle.System(meshgen.mesh2d(6), 1)
    coords, _, _ = s.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(2, 1, 4), coords)
    B = s.rhs(g)
    rp, col, val = s.A()
    val = -val
    X, its, rel, rs, st = oracle.pcg_csr(rp, col, val, B, 1e-10)
    assert st == -4
    # the healthy matrix through the same entry point agrees with the system call
    X1, its1, _, _, st1 = oracle.pcg_csr(*s.A(), B, 1e-10)
    X2, its2, _, _, st2 = s.pcg(B, 1e-10)
    assert st1 == st2 == 0 and np.array_equal(X1, X2) and its1[0] == its2[0]


def test_unreachable_tol_warns_after_the_last_restart():
    # below the rounding floor the true residual misses Eq. (2) after every
    # restart: status 1 (warning) with the residual reached, not success
    s = oracle.System(meshgen.mesh2d(12, 0.3, 2), 1)
    coords, _, _ = s.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(2, 1, 5), coords)
    X, its, rel, rs, st = s.pcg(s.rhs(g), 1e-17)
    assert st == 1 and rs[0] == 3 and rel[0] > 1e-17 and its[0] < oracle.default_max_iter(s.nfree)


def test_all_core_build_gives_the_serial_results():
    # the CPU baseline's all-core build runs the columns on separate threads;
    # each column keeps its arithmetic, so X, iterations and residuals equal
    # the one-thread oracle's bit for bit, a zero column included
    mesh = meshgen.make_mesh(3, 9, 0.2, 21)
    s = oracle.System(mesh, 1)
    coords, _, _ = s.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(3, 7, 22), coords)
    B = s.rhs(g)
    B[:, 3] = 0.0
    rp, col, val = s.A()
    ref = oracle.pcg_csr(rp, col, val, B, 1e-10)
    got = oracle.pcg_csr(rp, col, val, B, 1e-10, threads=4)
    assert ref[4] == got[4] == 0
    for a, b in zip(ref[:4], got[:4]):
        assert np.array_equal(a, b)
    assert ref[1][3] == 0 and np.all(ref[0][:, 3] == 0.0)
    assert oracle.omp_threads() >= 1
