"""pcg_tune through the C ABI: the report is consistent with the choice it
makes (FP64 fallback exactly when no mixed solve was faster), the matrix keeps
the tuned format, tiling and lanes per row, and a solve with the tuned
options passes the oracle's Eq. (2) check."""
import numpy as np
import pytest

import meshgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2201_05413_amd import femcg  # noqa: E402


# (dim, m, jitter, order, k): phase kernels with kp = 4 on P2, the one-column
# split-row candidates on P4, and a system small enough for the
# single-workgroup loop
@pytest.mark.parametrize("dim,m,jit,order,k", [(2, 120, 0.3, 2, 3), (2, 40, 0.25, 4, 1), (2, 30, 0.3, 1, 1)])
def test_tuned_options_solve_to_tol(dim, m, jit, order, k):
    tol = 1e-9
    mesh = meshgen.make_mesh(dim, m, jit, 31)
    orc = oracle.System(mesh, order)
    A = femcg.Matrix(mesh, order, femcg.FEM_FORMAT_SELL)
    coords, _, _ = A.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(dim, k, 32), coords)
    B = torch.empty((A.n_free, k), dtype=torch.float64, device="cuda")
    femcg.fem_rhs(A, g, B)
    opts, rep = femcg.pcg_tune(A, B, tol, femcg.default_opts(tol=tol, check_every=16))
    assert rep["format"] in (femcg.FEM_FORMAT_CSR, femcg.FEM_FORMAT_SELL)
    assert rep["lpr"] in ((1, 2, 4, 8) if k == 1 else (1,))
    assert rep["band"] in (0, 1, 2) and rep["ntiles"] >= 1
    if A.n_free * k <= 4096:
        assert rep["band"] == 2
    assert rep["fp64_ms"] > 0
    if rep["fp64_fallback"]:
        assert opts.precision == femcg.PCG_FP64
        assert rep["inner_eta"] == 0 or rep["mixed_ms"] >= rep["fp64_ms"]
    else:
        assert opts.precision == femcg.PCG_MIXED and rep["mixed_ms"] < rep["fp64_ms"]
        assert opts.inner_eta == rep["inner_eta"]
    assert rep["inner_eta"] in (0.0, 1e-2, 1e-3, 1e-4, 1e-5)
    # the tuned options, on the tuned matrix, reach tol by the oracle's check
    for prec in (opts.precision, femcg.PCG_FP64, femcg.PCG_MIXED):
        o = femcg.default_opts(tol=tol, check_every=16, precision=prec,
                               inner_eta=rep["inner_eta"] or 1e-4)
        X = torch.zeros_like(B)
        assert femcg.pcg_solve(A, B, X, tol, o) == 0
        torch.cuda.synchronize()
        assert np.all(orc.relres(orc.rhs(g), X.cpu().numpy()) <= tol * 1.0001)
    st = A.stats()
    assert st["format"] == rep["format"]
