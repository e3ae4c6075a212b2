"""Pins of the oracle's assembly, lifting and counts.

* structured 2D P1 (right-triangle split) is the 5-point stencil (4, -1), and
  the structured 3D Kuhn P1 matrix is h times the 7-point stencil (6, -1) --
  the paper's regular-grid matrix with w(i,j) = 1 (Sect. 2.2);
* the paper's Table 1 nonzero counts are reproduced by the 7-point stencil
  with one identity row per Dirichlet node;
* Table 7 counts the structural P1 pattern: nnz = V + 2E, and P2 DOFs = V + E;
* patch tests: P1 reproduces linear data and P2 reproduces x^2 - y^2 (both
  harmonic and inside the discrete space), so the lifted solution equals the
  data at every free DOF;
* the full stiffness is symmetric with zero row sums before Dirichlet
  conditions.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _csr(rp, col, val, n):
    return sp.csr_matrix((val, col, rp), shape=(n, n))


def _prune(M, rel=4 * np.finfo(float).eps):
    M = M.tocsr(copy=True)
    rowmax = np.maximum.reduceat(np.abs(M.data), M.indptr[:-1]) if M.nnz else np.zeros(0)
    rm = np.repeat(rowmax, np.diff(M.indptr))
    M.data[np.abs(M.data) <= rel * rm] = 0.0
    M.eliminate_zeros()
    return M


def _lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])


def test_structured_2d_p1_is_5_point_stencil():
    m = 20
    s = oracle.System(meshgen.mesh2d(m), 1)
    A = _prune(_csr(*s.A(), s.nfree))
    n = m - 2
    I = sp.identity(n)
    ref = (sp.kron(I, _lap1d(n)) + sp.kron(_lap1d(n), I)).tocsr()
    assert np.abs((A - ref).toarray()).max() <= 1e-14


def test_structured_3d_kuhn_p1_is_h_times_7_point_stencil():
    m = 9
    h = 1.0 / (m - 1)
    s = oracle.System(meshgen.mesh3d(m), 1)
    A = _prune(_csr(*s.A(), s.nfree))
    n = m - 2
    I = sp.identity(n)
    L = _lap1d(n)
    ref = h * (sp.kron(sp.kron(I, I), L) + sp.kron(sp.kron(I, L), I) + sp.kron(sp.kron(L, I), I))
    assert np.abs((A - ref).toarray()).max() <= 1e-14
    # structural pattern keeps 15 entries per interior row, 8 of them zero
    rp, _, _ = s.A()
    assert np.diff(rp).max() == 15


def test_table1_counts_reproduced_by_7_point_identity_rows():
    gold = json.load(open(os.path.join(GOLD, "table1_cube_nnz.json")))
    for c in gold["cubes"]:
        assert c["m"] ** 3 == c["rows"]
        assert oracle.fd7_identity_nnz(c["m"]) == c["nnz"], c["name"]


def _edges(cells):
    d = cells.shape[1]
    pairs = []
    for a in range(d):
        for b in range(a + 1, d):
            lo = np.minimum(cells[:, a], cells[:, b])
            hi = np.maximum(cells[:, a], cells[:, b])
            pairs.append(lo.astype(np.int64) * (1 << 32) + hi)
    return np.unique(np.concatenate(pairs))


def test_table7_count_conventions():
    gold = json.load(open(os.path.join(GOLD, "table7_counts.json")))
    V = gold["V"]
    E = gold["P2"]["dofs"] - V
    assert V + 2 * E == gold["P1"]["nnz"]
    mesh = meshgen.mesh2d(17, 0.3, 9)
    nv = mesh.nverts
    ne = len(_edges(mesh["cells"]))
    s1 = oracle.System(mesh, 1)
    s2 = oracle.System(mesh, 2)
    assert s1.nnz_K == nv + 2 * ne
    assert s2.ndofs == nv + ne


@pytest.mark.parametrize("dim,order,m,jit", [(2, 1, 13, 0.3), (3, 1, 7, 0.3), (2, 2, 9, 0.25),
                                             (3, 2, 5, 0.2)])
def test_stiffness_symmetric_zero_row_sums(dim, order, m, jit):
    s = oracle.System(meshgen.make_mesh(dim, m, jit, 3), order)
    K = _csr(*s.K(), s.ndofs)
    sc = np.abs(K.data).max()
    assert abs(K - K.T).max() <= 1e-14 * sc
    assert np.abs(np.asarray(K.sum(1))).max() <= 1e-13 * sc


@pytest.mark.parametrize("dim,order,m,jit,terms", [
    (2, 1, 15, 0.3, {0: 1.0, 1: 2.0, 2: -3.0}),
    (3, 1, 7, 0.3, {0: 0.5, 1: 1.0, 2: -2.0, 3: 0.25}),
    (2, 2, 11, 0.25, {3: 1.0}),
    (3, 2, 5, 0.2, {7: 1.0, 4: 0.5}),
])
def test_patch_exact_discrete_solution(dim, order, m, jit, terms):
    mesh = meshgen.make_mesh(dim, m, jit, 5)
    s = oracle.System(mesh, order)
    coords, dirich, f2d = s.dofs()
    co = meshgen.fixed_coeffs(dim, terms)
    g = meshgen.harmonic_eval(co, coords)
    # interior rows of K g vanish
    K = _csr(*s.K(), s.ndofs)
    Kg = K @ g[:, 0]
    assert np.abs(Kg[f2d]).max() <= 1e-12 * np.abs(K.data).max()
    B = s.rhs(g)
    X, its, rel, rs, st = s.pcg(B, 1e-13)
    assert st == 0
    assert oracle.x_err(g[f2d], X) <= 1e-10


def test_p2_dirichlet_edges_lie_on_the_boundary():
    for dim, m in [(2, 9), (3, 5)]:
        mesh = meshgen.make_mesh(dim, m, 0.2, 2)
        s = oracle.System(mesh, 2)
        coords, dirich, _ = s.dofs()
        on_bnd = np.any((np.abs(coords) < 1e-15) | (np.abs(coords - 1) < 1e-15), axis=1)
        assert np.array_equal(dirich.astype(bool), on_bnd)


def test_lifting_matches_dense_elimination():
    mesh = meshgen.mesh2d(9, 0.3, 4)
    s = oracle.System(mesh, 2)
    coords, dirich, f2d = s.dofs()
    K = _csr(*s.K(), s.ndofs).toarray()
    D = np.nonzero(dirich)[0]
    g = meshgen.harmonic_eval(meshgen.random_coeffs(2, 3, 7), coords)
    B = s.rhs(g)
    ref = -K[np.ix_(f2d, D)] @ g[D]
    assert np.abs(B - ref).max() <= 1e-13 * np.abs(ref).max()
    A = _csr(*s.A(), s.nfree).toarray()
    assert np.array_equal(A, K[np.ix_(f2d, f2d)])
