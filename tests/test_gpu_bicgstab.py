"""GPU parity of BiCGStab + Block-Jacobi (Sect. 3.2's solver) against the
oracle, through the C ABI (bicgstab_solve).

Bars: (R) the oracle recomputes ||b - A x|| / ||b|| with its own A: <= tol;
(S) at tol 1e-12 the solution is within 1e-8 relative L2 of the oracle's
PCG solution at 1e-14; iterations within 10% + 3 of the oracle's BiCGStab at
the same tolerance and block size (the recurrences round differently, and
BiCGStab's iteration count is more sensitive to rounding than CG's).
"""
import numpy as np
import pytest

import meshgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2201_05413_amd import femcg  # noqa: E402


class Sys:
    def __init__(self, dim, m, jit, order, seed=1, fmt=femcg.FEM_FORMAT_SELL):
        self.mesh = meshgen.make_mesh(dim, m, jit, seed)
        self.orc = oracle.System(self.mesh, order)
        self.A = femcg.Matrix(self.mesh, order, fmt)
        coords, _, self.f2d = self.orc.dofs()
        g = meshgen.harmonic_eval(meshgen.random_coeffs(dim, 1, seed + 100), coords)
        self.g = g + meshgen.noise(seed + 200, g.size, 0.01).reshape(g.shape)
        self.b = self.orc.rhs(self.g)[:, 0]
        self.rp, self.col, self.val = self.orc.A()

    def solve(self, tol, bs, max_iter=0):
        B = torch.empty((self.A.n_free, 1), dtype=torch.float64, device="cuda")
        femcg.fem_rhs(self.A, self.g, B)
        X = torch.full_like(B, 7.0)  # overwritten: the solve starts from zero
        rc, st = femcg.bicgstab_solve(self.A, B, X, tol, bs, max_iter)
        torch.cuda.synchronize()
        return rc, X.cpu().numpy()[:, 0], st


CASES = [(2, 45, 0.3, 1), (2, 21, 0.25, 2), (3, 11, 0.3, 1), (3, 7, 0.2, 2), (2, 13, 0.25, 4)]


@pytest.mark.parametrize("dim,m,jit,order", CASES)
@pytest.mark.parametrize("bs", [1, 4, 16, 64])
def test_bicgstab_matches_oracle(dim, m, jit, order, bs):
    c = Sys(dim, m, jit, order, seed=3)
    assert c.A.n_free % bs != 0 or bs == 1  # ragged last block
    Xs, _, _, _, st = c.orc.pcg(c.b[:, None], 1e-14)
    assert st == 0
    for tol in (1e-8, 1e-12):
        rc, x, stats = c.solve(tol, bs)
        assert rc == 0, stats
        rel = c.orc.relres(c.b[:, None], x[:, None])[0]
        # the library's own true residual agrees up to rounding noise
        assert rel <= tol * 1.0001 and abs(stats["relres"] - rel) <= 0.05 * rel + 1e-14, (rel, stats)
        assert stats["block_size"] == bs and stats["nblocks"] == -(-c.A.n_free // bs)
        _, its_o, rel_o, _, st_o = oracle.bicgstab_csr(c.rp, c.col, c.val, c.b, bs, tol)
        assert st_o == 0
        assert abs(stats["iters"] - its_o) <= 0.1 * its_o + 3, (stats["iters"], its_o)
        if tol == 1e-12:
            assert oracle.x_err(Xs[:, 0], x) <= 1e-8


@pytest.mark.parametrize("fmt,order_flag,C,sigma", [(femcg.FEM_FORMAT_CSR, 0, 64, 1),
                                                    (femcg.FEM_FORMAT_SELL, 0, 32, 1024),
                                                    (femcg.FEM_FORMAT_SELL, femcg.FEM_ORDER_SFC, 64, 64)])
def test_bicgstab_independent_of_the_internal_row_order(fmt, order_flag, C, sigma):
    # blocks are public rows; the solver copy's permutation must not change them
    c = Sys(2, 33, 0.3, 2, seed=5)
    femcg.fem_set_format(c.A, fmt | order_flag, C, sigma)
    rc, x, st = c.solve(1e-10, 8)
    assert rc == 0
    assert c.orc.relres(c.b[:, None], x[:, None])[0] <= 1e-10 * 1.0001
    _, its_o, _, _, _ = oracle.bicgstab_csr(c.rp, c.col, c.val, c.b, 8, 1e-10)
    assert abs(st["iters"] - its_o) <= 0.1 * its_o + 3


@pytest.mark.parametrize("dim,order", [(2, 2), (3, 2)])
def test_bicgstab_on_a_device_assembled_matrix(dim, order):
    c = Sys(dim, 30 if dim == 2 else 9, 0.2, order, seed=9, fmt=femcg.FEM_FORMAT_SELL | femcg.FEM_ASSEMBLE_DEVICE)
    rc, x, st = c.solve(1e-10, 16)
    assert rc == 0
    assert c.orc.relres(c.b[:, None], x[:, None])[0] <= 1e-10 * 1.0001


def test_one_block_is_exact_after_one_iteration():
    c = Sys(2, 8, 0.2, 1, seed=6)  # 36 free DOFs: one block of 64
    assert c.A.n_free <= 64
    rc, x, st = c.solve(1e-12, 64)
    assert rc == 0 and st["iters"] == 1 and st["nblocks"] == 1
    A = np.zeros((c.A.n_free, c.A.n_free))
    for i in range(c.A.n_free):
        A[i, c.col[c.rp[i]:c.rp[i + 1]]] = c.val[c.rp[i]:c.rp[i + 1]]
    xs = np.linalg.solve(A, c.b)
    assert np.abs(x - xs).max() <= 1e-12 * np.abs(xs).max()


def test_bicgstab_edge_cases():
    c = Sys(2, 20, 0.3, 1, seed=7)
    n = c.A.n_free
    B = torch.zeros((n, 1), dtype=torch.float64, device="cuda")
    X = torch.ones_like(B)
    rc, st = femcg.bicgstab_solve(c.A, B, X, 1e-10, 4)
    assert rc == 0 and st["iters"] == 0 and not X.cpu().numpy().any()
    # iteration cap: warning with the residual reached
    rc, x, st = c.solve(1e-12, 1, max_iter=5)
    assert rc == femcg.FEMCG_WARN_MAXITER and st["iters"] == 5 and st["relres"] > 1e-12
    # argument errors leave the matrix usable
    for bs in (0, 65):
        with pytest.raises(femcg.FemcgError) as ei:
            femcg.bicgstab_solve(c.A, B, X, 1e-10, bs)
        assert ei.value.code == femcg.FEMCG_EINVAL
    for tol in (0.0, -1.0, float("nan")):
        with pytest.raises(femcg.FemcgError) as ei:
            femcg.bicgstab_solve(c.A, B, X, tol, 4)
        assert ei.value.code == femcg.FEMCG_EINVAL
    Bn = torch.ones((n, 1), dtype=torch.float64, device="cuda")
    Bn[3, 0] = float("nan")
    with pytest.raises(femcg.FemcgError) as ei:
        femcg.bicgstab_solve(c.A, Bn, X, 1e-10, 4)
    assert ei.value.code == femcg.FEMCG_EBREAKDOWN
    rc, x, st = c.solve(1e-10, 4)
    assert rc == 0 and c.orc.relres(c.b[:, None], x[:, None])[0] <= 1e-10 * 1.0001
    # the PCG path still works on the same matrix
    Bp = torch.empty((n, 1), dtype=torch.float64, device="cuda")
    femcg.fem_rhs(c.A, c.g, Bp)
    Xp = torch.zeros_like(Bp)
    assert femcg.pcg_solve(c.A, Bp, Xp, 1e-10) == 0
