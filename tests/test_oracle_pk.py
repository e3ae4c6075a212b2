"""Pins of the oracle's P3/P4 triangles (Table 7's degrees 3 and 4).

* element: u^T K v for every pair of monomials x^p y^q (p + q <= k), taken at
  the element's lattice points, equals the exact integral of grad u . grad v
  over a general triangle, computed here in rational arithmetic (sympy) with
  the closed-form moments of the reference triangle -- no quadrature, no
  Vandermonde matrix;
* counts: DOFs = V + (k-1) E + (k-1)(k-2)/2 T, and the structural nonzeros
  follow from counting, for each DOF, the DOFs of the cells around it.  At
  the mesh counts that Table 7's DOF column fixes (V, E, T; the disk-like mesh
  then has 2E - 3T boundary edges) the count formula gives the printed P4
  nonzeros exactly;
* patch tests: Pk reproduces a harmonic polynomial of degree k at every DOF,
  and a degree k+1 one it does not;
* Dirichlet DOFs are exactly the DOFs on the boundary of the square.
"""
import json
import math
import os

import numpy as np
import pytest
import sympy

import meshgen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# element
# ---------------------------------------------------------------------------

def _exact_gram(Xr, k):
    """G[a][b] = integral over the triangle Xr (rationals) of grad m_a . grad m_b,
    m = x^p y^q with p + q <= k, by the pull-back to the unit right triangle
    and its moments  integral xi^i eta^j = i! j! / (i + j + 2)!."""
    x, y, s, t = sympy.symbols("x y s t")
    mons = [x ** (d - q) * y ** q for d in range(k + 1) for q in range(d + 1)]
    (x0, y0), (x1, y1), (x2, y2) = Xr
    det = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
    sub = {x: x0 + (x1 - x0) * s + (x2 - x0) * t, y: y0 + (y1 - y0) * s + (y2 - y0) * t}
    grads = [(sympy.diff(m, x), sympy.diff(m, y)) for m in mons]
    n = len(mons)
    G = np.zeros((n, n))
    for a in range(n):
        for b in range(a, n):
            f = sympy.Poly(sympy.expand((grads[a][0] * grads[b][0] + grads[a][1] * grads[b][1]).subs(sub)), s, t)
            val = sum(c * sympy.Rational(math.factorial(i) * math.factorial(j), math.factorial(i + j + 2))
                      for (i, j), c in f.terms())
            G[a, b] = G[b, a] = float(abs(det) * val)
    return mons, G


@pytest.mark.parametrize("k", [3, 4])
def test_pk_element_equals_exact_monomial_integrals(k):
    R = sympy.Rational
    Xr = [(R(1, 4), R(-1, 2)), (R(3, 2), R(1, 4)), (R(1, 2), R(7, 4))]  # exact in binary
    X = np.array([[float(c) for c in p] for p in Xr])
    K = oracle.pk_element(X, k)
    lp = oracle.pk_local_points(k)
    pts = (lp[:, 0:1] * X[0] + lp[:, 1:2] * X[1] + lp[:, 2:3] * X[2]) / k
    mons = [(d - q, q) for d in range(k + 1) for q in range(d + 1)]
    U = np.array([[px ** p * py ** q for (p, q) in mons] for px, py in pts])
    _, G = _exact_gram(Xr, k)
    assert np.abs(U.T @ K @ U - G).max() <= 1e-11 * np.abs(G).max()


@pytest.mark.parametrize("k", [3, 4])
def test_pk_element_properties(k):
    rng = np.random.default_rng(11 + k)
    X = rng.uniform(-1, 1, size=(3, 2))
    if np.linalg.det((X[1:] - X[0]).T) < 0:
        X = X[[0, 2, 1]]
    K = oracle.pk_element(X, k)
    nl = (k + 1) * (k + 2) // 2
    sc = np.abs(K).max()
    assert K.shape == (nl, nl)
    assert np.abs(K - K.T).max() <= 1e-14 * sc
    assert np.abs(K.sum(1)).max() <= 1e-12 * sc
    ev = np.linalg.eigvalsh(K)
    assert abs(ev[0]) <= 1e-12 * sc and ev[1] > 1e-6 * sc  # kernel = constants
    # invariance under a rigid motion and scaling by h: K scales by h^0 in 2D
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    K2 = oracle.pk_element(3.0 * X @ Rm.T + np.array([5.0, -2.0]), k)
    assert np.abs(K2 - K).max() <= 1e-11 * sc


def test_pk_degenerate_and_bad_degree_rejected():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0]])
    with pytest.raises(RuntimeError):
        oracle.pk_element(X, 3)
    with pytest.raises(RuntimeError):
        oracle.pk_element(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), 5)


# ---------------------------------------------------------------------------
# counts
# ---------------------------------------------------------------------------

def pk_dofs(k, V, E, T):
    return V + (k - 1) * E + (k - 1) * (k - 2) // 2 * T


def pk_structural_nnz(k, V, E, T, Eb):
    """Ordered pairs of DOFs sharing a triangle.  Row of a vertex of degree d
    in t triangles: 1 + d vertices, (k-1)(d + t) edge DOFs, ci t interior DOFs
    (sum d = 2E, sum t = 3T); row of an edge DOF: 2 nl - (k+1) on an interior
    edge, nl on a boundary edge; row of an interior DOF: nl."""
    nl = (k + 1) * (k + 2) // 2
    ci = (k - 1) * (k - 2) // 2
    Ei = E - Eb
    vert = V + 2 * E + (k - 1) * (2 * E + 3 * T) + ci * 3 * T
    edge = (k - 1) * (Ei * (2 * nl - (k + 1)) + Eb * nl)
    return vert + edge + ci * T * nl


def _mesh_counts(mesh):
    cells = np.asarray(mesh["cells"], dtype=np.int64)
    pairs = np.concatenate([np.sort(cells[:, [a, b]], axis=1) for a, b in [(0, 1), (0, 2), (1, 2)]])
    _, cnt = np.unique(pairs[:, 0] * (1 << 32) + pairs[:, 1], return_counts=True)
    return mesh.nverts, len(cnt), cells.shape[0], int((cnt == 1).sum())


@pytest.mark.parametrize("m,jit", [(6, 0.0), (9, 0.3)])
def test_pk_counts_match_formulas(m, jit):
    mesh = meshgen.mesh2d(m, jit, 4)
    V, E, T, Eb = _mesh_counts(mesh)
    for k in (1, 2, 3, 4):
        s = oracle.System(mesh, k)
        assert s.ndofs == pk_dofs(k, V, E, T)
        assert s.nnz_K == pk_structural_nnz(k, V, E, T, Eb), k


def test_table7_p3_p4_counts():
    g = json.load(open(os.path.join(GOLD, "table7_counts.json")))
    V = g["V"]
    E = g["P2"]["dofs"] - V
    T = g["P3"]["dofs"] - V - 2 * E
    assert V - E + T == 1  # Euler characteristic of a disk
    Eb = 2 * E - 3 * T
    assert Eb > 0
    assert pk_structural_nnz(1, V, E, T, Eb) == g["P1"]["nnz"]
    assert pk_dofs(4, V, E, T) == g["P4"]["dofs"]
    assert pk_structural_nnz(4, V, E, T, Eb) == g["P4"]["nnz"]


# ---------------------------------------------------------------------------
# patch tests and boundary
# ---------------------------------------------------------------------------

def _harm(deg, coords):
    z = coords[:, 0] + 1j * coords[:, 1]
    return (z ** deg).real[:, None] + 0.5 * (z ** (deg - 1)).imag[:, None]


@pytest.mark.parametrize("k,m,jit", [(3, 7, 0.25), (4, 6, 0.25)])
def test_pk_patch_reproduces_degree_k(k, m, jit):
    mesh = meshgen.mesh2d(m, jit, 5)
    s = oracle.System(mesh, k)
    coords, dirich, f2d = s.dofs()
    g = _harm(k, coords)
    X, its, rel, rs, st = s.pcg(s.rhs(g), 1e-14)
    assert st == 0
    assert oracle.x_err(g[f2d], X) <= 1e-10
    g2 = _harm(k + 1, coords)
    X2, _, _, _, st2 = s.pcg(s.rhs(g2), 1e-14)
    assert st2 == 0
    assert oracle.x_err(g2[f2d], X2) > 1e-6


def test_pk_smooth_error_decreases_with_degree():
    mesh = meshgen.mesh2d(7, 0.25, 6)
    errs = []
    for k in (1, 2, 3, 4):
        s = oracle.System(mesh, k)
        coords, _, f2d = s.dofs()
        g = (np.exp(coords[:, 0]) * np.cos(coords[:, 1]))[:, None]
        X, _, _, _, st = s.pcg(s.rhs(g), 1e-14)
        assert st == 0
        errs.append(np.abs(X[:, 0] - g[f2d, 0]).max())
    assert errs[0] > errs[1] > errs[2] > errs[3]


@pytest.mark.parametrize("k", [3, 4])
def test_pk_dirichlet_dofs_lie_on_the_boundary(k):
    mesh = meshgen.mesh2d(8, 0.2, 2)
    s = oracle.System(mesh, k)
    coords, dirich, _ = s.dofs()
    on_bnd = np.any((np.abs(coords) < 1e-15) | (np.abs(coords - 1) < 1e-15), axis=1)
    assert np.array_equal(dirich.astype(bool), on_bnd)
