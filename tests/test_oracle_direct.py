"""Pins of the oracle's dense Cholesky (Sect. 4.3's direct solver: factorise
once, forward and backward substitution per right-hand side), and of the
library's host-only nested-dissection analysis.

* the (2, -1) tridiagonal matrix has the closed-form factor
  L_ii = sqrt((i + 2) / (i + 1)), L_{i+1,i} = -sqrt((i + 1) / (i + 2));
* on FEM matrices, L is lower triangular with a positive diagonal and
  L L^T = A (the Cholesky factor is unique, so this fixes L);
* the solve recovers a known solution and agrees with the oracle's PCG at
  1e-14 (an independent method); an indefinite matrix reports breakdown;
* the nested-dissection order is a permutation, and the multifrontal entry
  count bounds the exact fill of that order from above.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle


def _csr(s):
    rp, col, val = s.A()
    return rp, col, val, sp.csr_matrix((val, col, rp), shape=(s.nfree, s.nfree))


def test_tridiagonal_closed_form():
    n = 40
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    _, L, st = oracle.dense_cholesky(A.indptr.astype(np.int64), A.indices, A.data, want_L=True)
    assert st == 0
    i = np.arange(n)
    assert np.allclose(np.diag(L), np.sqrt((i + 2) / (i + 1)), rtol=0, atol=1e-14)
    assert np.allclose(np.diag(L, -1), -np.sqrt((i[:-1] + 1) / (i[:-1] + 2)), rtol=0, atol=1e-14)
    assert np.all(np.triu(L, 1) == 0)


@pytest.mark.parametrize("dim,m,jit,order", [(2, 16, 0.3, 1), (2, 9, 0.25, 2), (3, 7, 0.3, 1), (3, 5, 0.2, 2)])
def test_factor_reproduces_A_and_solves(dim, m, jit, order):
    s = oracle.System(meshgen.make_mesh(dim, m, jit, 41), order)
    rp, col, val, A = _csr(s)
    Ad = A.toarray()
    rng = np.random.default_rng(42)
    Xt = rng.standard_normal((s.nfree, 3))
    B = A @ Xt
    X, L, st = oracle.dense_cholesky(rp, col, val, B, want_L=True)
    assert st == 0
    assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) > 0)
    assert np.abs(L @ L.T - Ad).max() <= 1e-13 * np.abs(Ad).max()
    assert np.linalg.norm(X - Xt) / np.linalg.norm(Xt) <= 1e-10
    # an independent method: the oracle's PCG at 1e-14
    g = meshgen.harmonic_eval(meshgen.random_coeffs(dim, 2, 43), s.dofs()[0])
    Bg = s.rhs(g)
    Xd, _, _ = oracle.dense_cholesky(rp, col, val, Bg)
    Xp, _, _, _, stp = s.pcg(Bg, 1e-14)
    assert stp == 0
    assert np.linalg.norm(Xd - Xp) / np.linalg.norm(Xp) <= 1e-10


def test_indefinite_matrix_breaks_down():
    s = oracle.System(meshgen.make_mesh(2, 10, 0.2, 44), 1)
    rp, col, val, _ = _csr(s)
    val = val.copy()
    for t in range(rp[5], rp[6]):
        if col[t] == 5:
            val[t] = -val[t]
    _, _, st = oracle.dense_cholesky(rp, col, val, np.ones(s.nfree))
    assert st == -4


def _exact_fill(Ap):
    """Entries of the Cholesky factor of the pattern Ap (boolean, symmetric),
    by symbolic elimination: column j's structure joins every later column
    it reaches."""
    n = Ap.shape[0]
    S = np.tril(Ap).astype(bool)
    for j in range(n):
        rows = np.nonzero(S[j + 1:, j])[0] + j + 1
        for a in rows:
            S[rows[rows >= a], a] = True
    return int(S.sum())


@pytest.mark.parametrize("dim,m,jit,order", [(2, 22, 0.3, 1), (3, 8, 0.2, 1), (2, 10, 0.25, 2)])
def test_host_analysis_orders_and_bounds_fill(dim, m, jit, order):
    from paper_2201_05413_amd import femcg
    mesh = meshgen.make_mesh(dim, m, jit, 45)
    H = femcg.Matrix(mesh, order, femcg.FEM_FORMAT_CSR | femcg.FEM_ASSEMBLE_HOST_ONLY)
    st, perm = femcg.chol_analyze(H)
    n = H.n_free
    assert st["n"] == n and np.array_equal(np.sort(perm), np.arange(n))
    s = oracle.System(mesh, order)
    _, _, _, A = _csr(s)
    Ad = np.abs(A.toarray()) > 4 * 2.220446049250313e-16 * np.abs(A.toarray()).max(axis=1, keepdims=True)
    Ap = Ad[np.ix_(perm, perm)]
    exact = _exact_fill(Ap | Ap.T)
    assert exact <= st["nnz_l"] <= n * (n + 1) // 2
    assert st["max_front"] <= n and st["nodes"] >= 1 and st["flops"] > 0


def test_host_analysis_is_deterministic():
    # the ordering runs its top subtrees on threads of their own and the
    # update sets level by level in parallel: repeated analyses agree
    from paper_2201_05413_amd import femcg
    mesh = meshgen.make_mesh(3, 30, 0.2, 46)
    H = femcg.Matrix(mesh, 1, femcg.FEM_FORMAT_CSR | femcg.FEM_ASSEMBLE_HOST_ONLY)
    st0, p0 = femcg.chol_analyze(H)
    for _ in range(3):
        st, p = femcg.chol_analyze(H)
        assert np.array_equal(p, p0)
        assert (st["nnz_l"], st["nodes"], st["levels"], st["max_front"], st["flops"]) == \
            (st0["nnz_l"], st0["nodes"], st0["levels"], st0["max_front"], st0["flops"])
