"""Degenerate inputs and argument errors through the C ABI (host-side checks
and kernel-side breakdown flags); every path must return its error code and
leave the library usable."""
import numpy as np
import pytest

import meshgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2201_05413_amd import femcg  # noqa: E402


def test_mesh_without_free_dofs():
    mesh = meshgen.make_mesh(2, 2, 0.0, 1)  # 4 vertices, all on the boundary
    with pytest.raises(femcg.FemcgError) as ei:
        femcg.Matrix(mesh, 1)
    assert ei.value.code == femcg.FEMCG_EINVAL


@pytest.mark.parametrize("dim", [2, 3])
def test_inverted_cell_is_rejected(dim):
    mesh = dict(meshgen.make_mesh(dim, 6, 0.0, 1))
    cells = np.array(mesh["cells"], copy=True)
    cells[3, [0, 1]] = cells[3, [1, 0]]  # one cell with negative orientation
    mesh["cells"] = cells
    with pytest.raises(femcg.FemcgError) as ei:
        femcg.Matrix(mesh, 1)
    assert ei.value.code == femcg.FEMCG_EMESH


@pytest.mark.parametrize("dim,order", [(3, 3), (3, 4), (2, 5), (2, 0)])
def test_unsupported_order_is_rejected(dim, order):
    with pytest.raises(femcg.FemcgError) as ei:
        femcg.Matrix(meshgen.make_mesh(dim, 5, 0.0, 1), order)
    assert ei.value.code == femcg.FEMCG_EUNSUPPORTED


def test_argument_errors():
    mesh = meshgen.make_mesh(2, 12, 0.2, 1)
    A = femcg.Matrix(mesh, 1)
    n = A.n_free
    for k, code in ((65, femcg.FEMCG_EUNSUPPORTED), (0, femcg.FEMCG_EUNSUPPORTED)):
        B = torch.zeros((n, max(k, 1)), dtype=torch.float64, device="cuda")
        X = torch.zeros_like(B)
        rc = femcg.lib().pcg_solve(A.h, B.data_ptr(), X.data_ptr(), k, 1e-8, None, None)
        assert rc == code
    B = torch.ones((n, 1), dtype=torch.float64, device="cuda")
    X = torch.zeros_like(B)
    for tol in (0.0, -1.0, float("nan")):
        assert femcg.lib().pcg_solve(A.h, B.data_ptr(), X.data_ptr(), 1, tol, None, None) == femcg.FEMCG_EINVAL
    # still usable afterwards
    assert femcg.pcg_solve(A, B, X, 1e-10) == 0


@pytest.mark.parametrize("mode", [2, 0, 1])
@pytest.mark.parametrize("prec", [femcg.PCG_FP64, femcg.PCG_MIXED])
def test_nonfinite_rhs_column_is_a_breakdown(mode, prec):
    # a NaN in column 1 breaks that column down; column 0 still converges
    mesh = meshgen.make_mesh(2, 30, 0.3, 5)
    orc = oracle.System(mesh, 1)
    A = femcg.Matrix(mesh, 1)
    femcg.fem_set_tiling(A, mode, 0 if mode != 1 else 1024)
    coords, _, _ = orc.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(2, 2, 6), coords)
    B = torch.empty((A.n_free, 2), dtype=torch.float64, device="cuda")
    femcg.fem_rhs(A, g, B)
    B[7, 1] = float("nan")
    X = torch.zeros_like(B)
    with pytest.raises(femcg.FemcgError) as ei:
        femcg.pcg_solve(A, B, X, 1e-10, femcg.default_opts(tol=1e-10, precision=prec))
    torch.cuda.synchronize()
    assert ei.value.code == femcg.FEMCG_EBREAKDOWN
    x0 = X.cpu().numpy()[:, 0:1]
    assert np.all(orc.relres(orc.rhs(g[:, 0:1]), x0) <= 1e-10 * 1.0001)
