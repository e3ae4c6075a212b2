"""Pins of the oracle's element matrices.

Each element matrix K_ij = integral grad(phi_i).grad(phi_j) (Sect. 2.2's
Laplacian, sign flipped so K is PSD) is checked against constructions that
share nothing with the oracle's C code:

* P1: the paper's cotangent weights (Sect. 2.2) vs the gradient form;
* P1 and P2: a Lagrange basis built here from a monomial Vandermonde system,
  integrated with a collapsed (Duffy) tensor Gauss-Legendre rule of high degree;
* closed-form facts: symmetry, constants in the kernel (zero row sums),
  rank d, and the P2 coupling between a vertex and the midpoint of an edge
  away from it (zero on triangles, closed form on tetrahedra).
"""
import itertools

import numpy as np
import pytest

import oracle


def _rand_simplex(rng, dim):
    while True:
        X = rng.uniform(-1, 1, size=(dim + 1, dim))
        M = (X[1:] - X[0]).T
        if np.linalg.det(M) > 0.05:
            return X


def _nodes(X, order):
    dim = X.shape[1]
    if order == 1:
        return X.copy()
    pts = [X[i] for i in range(dim + 1)]
    for a, b in itertools.combinations(range(dim + 1), 2):
        pts.append(0.5 * (X[a] + X[b]))
    return np.array(pts)


def _monomials(dim, order):
    """exponent tuples of total degree <= order"""
    return [e for e in itertools.product(range(order + 1), repeat=dim) if sum(e) <= order]


def _lagrange_coeffs(X, order):
    dim = X.shape[1]
    mons = _monomials(dim, order)
    N = _nodes(X, order)
    V = np.array([[np.prod(p ** np.array(e)) for e in mons] for p in N])
    # phi_i = sum_m C[m, i] mon_m, with phi_i(node_j) = delta_ij
    return mons, np.linalg.solve(V, np.eye(len(N)))


def _grad_mon(e, p):
    g = np.zeros(len(e))
    for r in range(len(e)):
        if e[r] > 0:
            ee = list(e)
            ee[r] -= 1
            g[r] = e[r] * np.prod(p ** np.array(ee))
    return g


def _duffy_rule(dim, n=6):
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    pts, wts = [], []
    if dim == 2:
        for i in range(n):
            for j in range(n):
                u, v = x[i], x[j]
                pts.append((u, v * (1 - u)))
                wts.append(w[i] * w[j] * (1 - u))
    else:
        for i in range(n):
            for j in range(n):
                for l in range(n):
                    u, v, t = x[i], x[j], x[l]
                    pts.append((u, v * (1 - u), t * (1 - u) * (1 - v)))
                    wts.append(w[i] * w[j] * w[l] * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


def brute_stiffness(X, order):
    dim = X.shape[1]
    mons, Cf = _lagrange_coeffs(X, order)
    nl = Cf.shape[1]
    ref, wts = _duffy_rule(dim)
    M = (X[1:] - X[0]).T
    detJ = abs(np.linalg.det(M))
    K = np.zeros((nl, nl))
    for p_ref, w in zip(ref, wts):
        p = X[0] + M @ p_ref
        Gm = np.array([_grad_mon(e, p) for e in mons])  # [nmon][dim]
        G = Cf.T @ Gm                                   # [nl][dim]
        K += w * detJ * (G @ G.T)
    return K


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_gradient_equals_cotangent(dim):
    rng = np.random.default_rng(10 + dim)
    for _ in range(50):
        X = _rand_simplex(rng, dim)
        Kg = oracle.p1_element(X)
        Kc = oracle.p1_element_cot(X)
        assert np.abs(Kg - Kc).max() <= 1e-12 * np.abs(Kg).max()


@pytest.mark.parametrize("dim,order", [(2, 1), (3, 1), (2, 2), (3, 2)])
def test_element_matches_bruteforce_quadrature(dim, order):
    rng = np.random.default_rng(100 * dim + order)
    fn = oracle.p1_element if order == 1 else oracle.p2_element
    for _ in range(8):
        X = _rand_simplex(rng, dim)
        K = fn(X)
        Kb = brute_stiffness(X, order)
        assert np.abs(K - Kb).max() <= 1e-10 * np.abs(Kb).max()


@pytest.mark.parametrize("dim,order", [(2, 1), (3, 1), (2, 2), (3, 2)])
def test_element_closed_form_properties(dim, order):
    rng = np.random.default_rng(7 * dim + order)
    fn = oracle.p1_element if order == 1 else oracle.p2_element
    for _ in range(20):
        X = _rand_simplex(rng, dim)
        K = fn(X)
        sc = np.abs(K).max()
        assert np.abs(K - K.T).max() <= 1e-14 * sc
        assert np.abs(K.sum(1)).max() <= 1e-13 * sc  # constants in the kernel
        ev = np.linalg.eigvalsh(0.5 * (K + K.T))
        assert ev[0] >= -1e-12 * sc and ev[1] > 1e-8 * sc  # PSD, kernel = constants


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_vertex_opposite_midpoint_coupling(dim):
    # K[v, e] = 4 sum_{c in e} grad(l_v).grad(l_c') * integral (4 l_v - 1) l_c,
    # and integral (4 l_v - 1) l_c = |T| (4/((d+1)(d+2)) - 1/(d+1)):
    # zero on triangles, -|T|/20 on tetrahedra
    rng = np.random.default_rng(55 + dim)
    edges = list(itertools.combinations(range(dim + 1), 2))
    for _ in range(20):
        X = _rand_simplex(rng, dim)
        K = oracle.p2_element(X)
        sc = np.abs(K).max()
        for v in range(dim + 1):
            for e, (a, b) in enumerate(edges):
                if v not in (a, b):
                    if dim == 2:
                        assert abs(K[v, dim + 1 + e]) <= 1e-14 * sc
                    else:
                        M = (X[1:] - X[0]).T
                        vol = np.linalg.det(M) / 6.0
                        Gi = np.linalg.inv(M)  # rows: grad l_1..l_3
                        G = np.vstack([-Gi.sum(0), Gi])
                        ref = 4 * (-vol / 20.0) * (G[v] @ G[b] + G[v] @ G[a])
                        assert abs(K[v, dim + 1 + e] - ref) <= 1e-12 * sc


def test_reference_triangle_values():
    # unit right triangle: the textbook P1 matrix [[1,-.5,-.5],[-.5,.5,0],[-.5,0,.5]]
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    K = oracle.p1_element(X)
    ref = np.array([[1.0, -0.5, -0.5], [-0.5, 0.5, 0.0], [-0.5, 0.0, 0.5]])
    assert np.abs(K - ref).max() <= 1e-15


def test_degenerate_element_rejected():
    X = np.array([[0.0, 0.0], [0.0, 1.0], [1.0, 0.0]])  # negative orientation
    with pytest.raises(RuntimeError):
        oracle.p1_element(X)
