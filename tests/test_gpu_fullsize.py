"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (autotuned format, check_every 64, FP64 and mixed): the oracle's own
Eq. (2) residual of every column (R), and the closed forms where the exact
discrete solution is known (C3: nodal harmonic cubics on the structured
Kuhn mesh; C4 column 0: the P2 interpolant of x^2 - y^2), within the bound a
1e-8 residual allows.  BiCGStab + Block-Jacobi runs on the full C2 system
and on the full C3 cube."""
import numpy as np
import pytest

import meshgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from paper_2201_05413_amd import femcg  # noqa: E402


def _run(w):
    A = femcg.Matrix(w.mesh, w.order)
    coords, _, f2d = A.dofs()
    g = w.dirichlet(coords)
    B = torch.empty((A.n_free, w.k), dtype=torch.float64, device="cuda")
    femcg.fem_rhs(A, g, B)
    femcg.fem_tune(A, w.k, femcg.PCG_FP64)
    out = {}
    for prec in (femcg.PCG_FP64, femcg.PCG_MIXED):
        X = torch.zeros_like(B)
        rc = femcg.pcg_solve(A, B, X, w.tol, femcg.default_opts(tol=w.tol, precision=prec, check_every=64))
        torch.cuda.synchronize()
        assert rc == 0, (w.name, prec, A.stats())
        out[prec] = X.cpu().numpy()
    del B, A
    orc = oracle.System(w.mesh, w.order)
    Bo = orc.rhs(g)
    for prec, X in out.items():
        rel = orc.relres(Bo, X)
        assert np.all(rel <= w.tol * 1.0001), (w.name, prec, rel.max())
    return g, f2d, out


def test_c2_full_size():
    _run(meshgen.c2())


def test_c3_full_size_and_cubics():
    w = meshgen.c3()
    g, f2d, out = _run(w)
    for X in out.values():
        for j in range(w.k):
            assert oracle.x_err(g[f2d, j], X[:, j]) <= 1e-5


def test_c4_full_size_and_column0_closed_form():
    w = meshgen.c4()
    g, f2d, out = _run(w)
    for X in out.values():
        assert oracle.x_err(g[f2d, 0], X[:, 0]) <= 1e-5


@pytest.mark.parametrize("bs", [1, 4])
def test_c2_full_size_bicgstab(bs):
    # the paper's solver on the full C2 system (its lifted right-hand side
    # lives next to the boundary: the Lanczos restart path)
    w = meshgen.c2()
    A = femcg.Matrix(w.mesh, w.order)
    femcg.fem_tune(A, 1, femcg.PCG_FP64)
    coords, _, _ = A.dofs()
    g = w.dirichlet(coords)[:, :1].copy()
    B = torch.empty((A.n_free, 1), dtype=torch.float64, device="cuda")
    femcg.fem_rhs(A, g, B)
    X = torch.zeros_like(B)
    rc, st = femcg.bicgstab_solve(A, B, X, w.tol, bs)
    torch.cuda.synchronize()
    assert rc == 0, st
    orc = oracle.System(w.mesh, w.order)
    rel = orc.relres(orc.rhs(g), X.cpu().numpy())[0]
    assert rel <= w.tol * 1.0001, (rel, st)


@pytest.mark.parametrize("bs", [1, 4])
def test_c3_full_size_bicgstab(bs):
    # the paper's solver on the full 128^3 Kuhn cube (Cube 1's grid), column
    # 0 of C3's data: the oracle's residual (R), and the nodal harmonic cubic,
    # which is the exact discrete solution on this mesh
    w = meshgen.c3()
    A = femcg.Matrix(w.mesh, w.order)
    femcg.fem_tune(A, 1, femcg.PCG_FP64)
    coords, _, f2d = A.dofs()
    g = w.dirichlet(coords)[:, :1].copy()
    B = torch.empty((A.n_free, 1), dtype=torch.float64, device="cuda")
    femcg.fem_rhs(A, g, B)
    X = torch.zeros_like(B)
    rc, st = femcg.bicgstab_solve(A, B, X, w.tol, bs)
    torch.cuda.synchronize()
    assert rc == 0, st
    x = X.cpu().numpy()
    del B, X, A
    orc = oracle.System(w.mesh, w.order)
    rel = orc.relres(orc.rhs(g), x)[0]
    assert rel <= w.tol * 1.0001, (rel, st)
    assert oracle.x_err(g[f2d, 0], x[:, 0]) <= 1e-5


def test_c2_full_size_bicgstab_on_the_paper_form():
    # A = B^-1 L (Sect. 2.2) on the full C2 system: rows scaled by the inverse
    # area of the cells around each vertex; the oracle's matrix gives the
    # scaled residual
    import scipy.sparse as sp
    w = meshgen.c2()
    A = femcg.Matrix(w.mesh, w.order)
    femcg.fem_tune(A, 1, femcg.PCG_FP64)
    coords, _, f2d = A.dofs()
    Xc = np.asarray(w.mesh["coords"], dtype=np.float64)
    T = np.asarray(w.mesh["cells"], dtype=np.int64)
    area = 0.5 * np.abs((Xc[T[:, 1], 0] - Xc[T[:, 0], 0]) * (Xc[T[:, 2], 1] - Xc[T[:, 0], 1])
                        - (Xc[T[:, 2], 0] - Xc[T[:, 0], 0]) * (Xc[T[:, 1], 1] - Xc[T[:, 0], 1]))
    Bl = np.zeros(len(Xc))
    for j in range(3):
        np.add.at(Bl, T[:, j], area)
    dsc = 1.0 / Bl[f2d]
    g = w.dirichlet(coords)[:, :1].copy()
    B = torch.empty((A.n_free, 1), dtype=torch.float64, device="cuda")
    femcg.fem_rhs(A, g, B)
    X = torch.zeros_like(B)
    rc, st = femcg.bicgstab_solve(A, B, X, w.tol, 4, row_scale=dsc)
    torch.cuda.synchronize()
    assert rc == 0, st
    orc = oracle.System(w.mesh, w.order)
    rp, col, val = orc.A()
    Ao = sp.csr_matrix((val, col, rp), shape=(A.n_free, A.n_free))
    b = orc.rhs(g)[:, 0]
    x = X.cpu().numpy()[:, 0]
    rel = np.linalg.norm(dsc * (b - Ao @ x)) / np.linalg.norm(dsc * b)
    assert rel <= w.tol * 1.0001 and abs(st["relres"] - rel) <= 0.05 * rel, (rel, st)
