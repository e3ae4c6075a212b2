"""GPU parity of the HIP path against the oracle, through the C ABI.

Bars (see the oracle's pins for what fixes the oracle itself):
* assembly: identical structural pattern, max_row |dA| / max_row |A| <= 1e-12
  (P1..P4, host and device assembly);
  B = -K_ID g_D within 1e-12 norm-wise per column; DOF coordinates bit-equal;
* SpMM: |y - y_oracle| <= 1e-13 (|A| |x|) row-wise (FP64; the solver copy
  drops entries below 4 eps64 max_row|a|);
* solve (R): the oracle recomputes ||b - A x|| / ||b|| with its own A: <= tol;
* solve (S): at tol 1e-12 the solution is within 1e-8 relative L2 of the
  oracle's solution at tol 1e-14 (or of the closed form where one exists).
Sizes span several tiles and end in a ragged tail.
"""
import numpy as np
import pytest

import meshgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2201_05413_amd import femcg  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


class Case:
    def __init__(self, dim, m, jit, order, k, seed=1, fmt=femcg.FEM_FORMAT_SELL, noise=0.0):
        self.mesh = meshgen.make_mesh(dim, m, jit, seed)
        self.order = order
        self.k = k
        self.orc = oracle.System(self.mesh, order)
        self.A = femcg.Matrix(self.mesh, order, fmt)
        coords, _, self.f2d = self.orc.dofs()
        co = meshgen.random_coeffs(dim, k, seed + 100)
        self.g = meshgen.harmonic_eval(co, coords)
        if noise > 0:
            self.g = self.g + meshgen.noise(seed + 200, self.g.size, noise).reshape(self.g.shape)
        self.Bo = self.orc.rhs(self.g)

    def B(self):
        B = torch.empty((self.A.n_free, self.k), dtype=torch.float64, device="cuda")
        femcg.fem_rhs(self.A, self.g, B)
        return B

    def solve(self, tol, **kw):
        B = self.B()
        X = torch.zeros_like(B)
        o = femcg.default_opts(tol=tol, **kw)
        rc = femcg.pcg_solve(self.A, B, X, tol, o)
        torch.cuda.synchronize()
        return rc, X.cpu().numpy(), self.A.stats()


CASES = [
    (2, 37, 0.3, 1), (2, 23, 0.25, 2), (3, 11, 0.3, 1), (3, 7, 0.2, 2), (2, 64, 0.0, 1), (3, 17, 0.0, 1),
    # P3 / P4 triangles (Table 7's degrees 3 and 4): rows of up to 49 / 81
    # entries; the last one fits the single-workgroup loop
    (2, 17, 0.3, 3), (2, 13, 0.25, 4), (2, 6, 0.2, 4),
]


@pytest.mark.parametrize("dim,m,jit,order", CASES)
@pytest.mark.parametrize("where", [0, femcg.FEM_ASSEMBLE_DEVICE], ids=["host", "device"])
def test_assembly_matches_oracle(dim, m, jit, order, where):
    c = Case(dim, m, jit, order, 2, fmt=femcg.FEM_FORMAT_SELL | where)
    coords_l, dir_l, f2d_l = c.A.dofs()
    coords_o, dir_o, f2d_o = c.orc.dofs()
    assert np.array_equal(coords_l, coords_o)
    assert np.array_equal(dir_l, dir_o) and np.array_equal(f2d_l, f2d_o)
    rp, col, val = c.A.csr()
    rpo, colo, valo = c.orc.A()
    assert np.array_equal(rp, rpo) and np.array_equal(col, colo)
    rowmax = np.maximum.reduceat(np.abs(valo), rpo[:-1])
    dmax = np.maximum.reduceat(np.abs(val - valo), rpo[:-1])
    assert (dmax / rowmax).max() <= 1e-12
    B = c.B().cpu().numpy()
    for j in range(c.k):
        assert np.linalg.norm(B[:, j] - c.Bo[:, j]) <= 1e-12 * np.linalg.norm(c.Bo[:, j])


@pytest.mark.parametrize("fmt", [femcg.FEM_FORMAT_CSR, femcg.FEM_FORMAT_SELL])
@pytest.mark.parametrize("k", [1, 3, 8, 12, 16, 32, 64])
@pytest.mark.parametrize("order,m", [(2, 45), (4, 21)])
def test_spmm_matches_oracle(fmt, k, order, m):
    # P4 rows hold up to 81 entries: split rows at k = 1, vector lanes at k >= 8
    c = Case(2, m, 0.3, order, 1, seed=3, fmt=fmt)
    rng = np.random.default_rng(k)
    X = rng.standard_normal((c.A.n_free, k))
    Y = torch.zeros((c.A.n_free, k), dtype=torch.float64, device="cuda")
    femcg.fem_spmv(c.A, dev(X), Y)
    torch.cuda.synchronize()
    Yo = c.orc.spmv(X)
    rp, col, val = c.orc.A()
    absAx = np.zeros_like(X)
    for i in range(c.orc.nfree):
        absAx[i] = np.abs(val[rp[i]:rp[i + 1]]) @ np.abs(X[col[rp[i]:rp[i + 1]]])
    assert np.all(np.abs(Y.cpu().numpy() - Yo) <= 1e-13 * absAx)


@pytest.mark.parametrize("lpr", [None, 1, 2, 4, 8])
@pytest.mark.parametrize("order,m", [(3, 19), (4, 15)])
def test_k1_split_rows_match_oracle(order, m, lpr, monkeypatch):
    # k = 1 SpMM with the long P3/P4 rows split over 1, 2, 4 or 8 lanes
    # (None: the automatic choice), through fem_spmv and the phase kernels
    if lpr is not None:
        monkeypatch.setenv("FEMCG_LPR", str(lpr))
    c = Case(2, m, 0.3, order, 1, seed=5, noise=0.01)
    X = np.random.default_rng(order).standard_normal((c.A.n_free, 1))
    Y = torch.zeros((c.A.n_free, 1), dtype=torch.float64, device="cuda")
    femcg.fem_spmv(c.A, dev(X), Y)
    torch.cuda.synchronize()
    rp, col, val = c.orc.A()
    absAx = np.array([np.abs(val[rp[i]:rp[i + 1]]) @ np.abs(X[col[rp[i]:rp[i + 1]], 0])
                      for i in range(c.orc.nfree)])
    assert np.all(np.abs(Y.cpu().numpy()[:, 0] - c.orc.spmv(X)[:, 0]) <= 1e-13 * absAx)
    femcg.fem_set_tiling(c.A, 0, 0)
    _, its_t, _, _, _ = c.orc.pcg(c.Bo, 1e-10)
    rc, Xs, st = c.solve(1e-10)
    assert rc == 0, st
    assert np.all(c.orc.relres(c.Bo, Xs) <= 1e-10 * 1.0001)
    assert abs(st["iters"][0] - its_t[0]) <= 0.02 * its_t[0] + 2, (st["iters"], its_t)


@pytest.mark.parametrize("dim,m,jit,order", CASES)
@pytest.mark.parametrize("prec", [femcg.PCG_FP64, femcg.PCG_MIXED])
def test_solve_matches_oracle(dim, m, jit, order, prec):
    c = Case(dim, m, jit, order, 3, noise=0.01)
    Xs, its_o, _, _, st = c.orc.pcg(c.Bo, 1e-14)
    assert st == 0
    # (R) at tol 1e-8 and (S) at tol 1e-12
    for tol in (1e-8, 1e-12):
        rc, X, stats = c.solve(tol, precision=prec)
        assert rc == 0, stats
        rel = c.orc.relres(c.Bo, X)
        assert np.all(rel <= tol * 1.0001), (rel, stats)
        if tol == 1e-12:
            for j in range(c.k):
                assert oracle.x_err(Xs[:, j], X[:, j]) <= 1e-8
        if prec == femcg.PCG_FP64 and tol == 1e-8:
            _, its_t, _, _, _ = c.orc.pcg(c.Bo, tol)
            for j in range(c.k):
                assert abs(stats["iters"][j] - its_t[j]) <= 0.02 * its_t[j] + 2, (stats["iters"], its_t)


WIDE_K = [(2, 37, 0.3, 1, 12), (3, 11, 0.3, 1, 16), (2, 23, 0.25, 2, 64), (3, 9, 0.2, 2, 12)]


@pytest.mark.parametrize("dim,m,jit,order,k", WIDE_K)
@pytest.mark.parametrize("mode", [0, 1], ids=["tile", "band"])
@pytest.mark.parametrize("prec", [femcg.PCG_FP64, femcg.PCG_MIXED])
def test_wide_k_phase_kernels_match_oracle(dim, m, jit, order, k, mode, prec):
    # kp = 16 (k = 12, 16) and kp = 64 instances of the phase kernels, FP64
    # and FP32-inner, in tile mode and in band mode (small tiles, several
    # reduction groups): SpMM element by element, (R) at 1e-8, (S) at 1e-12
    c = Case(dim, m, jit, order, k, seed=43, noise=0.01)
    assert c.A.n_free * (16 if k <= 16 else 64) > 4096  # not the single-workgroup loop
    femcg.fem_set_tiling(c.A, mode, 1024 if mode == 1 else 0)
    rng = np.random.default_rng(k + mode)
    Xr = rng.standard_normal((c.A.n_free, k))
    Y = torch.zeros((c.A.n_free, k), dtype=torch.float64, device="cuda")
    femcg.fem_spmv(c.A, dev(Xr), Y)
    torch.cuda.synchronize()
    rp, col, val = c.orc.A()
    absAx = np.zeros_like(Xr)
    for i in range(c.orc.nfree):
        absAx[i] = np.abs(val[rp[i]:rp[i + 1]]) @ np.abs(Xr[col[rp[i]:rp[i + 1]]])
    assert np.all(np.abs(Y.cpu().numpy() - c.orc.spmv(Xr)) <= 1e-13 * absAx)
    Xs, _, _, _, st = c.orc.pcg(c.Bo, 1e-14)
    assert st == 0
    _, its_t, _, _, _ = c.orc.pcg(c.Bo, 1e-8)
    for tol in (1e-8, 1e-12):
        rc, X, stats = c.solve(tol, precision=prec)
        assert rc == 0, stats
        assert np.all(c.orc.relres(c.Bo, X) <= tol * 1.0001)
        if tol == 1e-12:
            for j in range(k):
                assert oracle.x_err(Xs[:, j], X[:, j]) <= 1e-8, j
        elif prec == femcg.PCG_FP64:
            for j in range(k):
                assert abs(stats["iters"][j] - its_t[j]) <= 0.02 * its_t[j] + 2, (stats["iters"], its_t)


def test_c1_closed_form():
    w = meshgen.c1()
    A = femcg.Matrix(w.mesh, 1)
    coords, _, f2d = A.dofs()
    g = w.dirichlet(coords)
    B = torch.empty((A.n_free, 1), dtype=torch.float64, device="cuda")
    femcg.fem_rhs(A, g, B)
    X = torch.zeros_like(B)
    assert femcg.pcg_solve(A, B, X, 1e-10) == 0
    x = X.cpu().numpy()
    assert oracle.x_err(g[f2d], x) <= 1e-9
    assert abs(A.stats()["iters"][0] - 197) <= 6


def test_structured_3d_harmonic_cubics_closed_form():
    c = Case(3, 24, 0.0, 1, 8, seed=3)
    for prec in (femcg.PCG_FP64, femcg.PCG_MIXED):
        rc, X, st = c.solve(1e-12, precision=prec)
        assert rc == 0
        for j in range(c.k):
            assert oracle.x_err(c.g[c.f2d, j], X[:, j]) <= 1e-8


def test_zero_rhs_column_and_odd_k():
    c = Case(2, 30, 0.3, 1, 5, seed=7)
    c.g[:, 2] = 0.0
    c.Bo = c.orc.rhs(c.g)
    rc, X, st = c.solve(1e-10)
    assert rc == 0
    assert st["iters"][2] == 0 and np.all(X[:, 2] == 0.0)
    rel = c.orc.relres(c.Bo, X)
    assert np.all(rel[[0, 1, 3, 4]] <= 1e-10)


def test_max_iter_warning_and_initial_guess():
    c = Case(2, 40, 0.3, 1, 1, seed=9)
    rc, X, st = c.solve(1e-10, max_iter=7, check_every=4)
    assert rc == femcg.FEMCG_WARN_MAXITER and st["iters"][0] == 7 and st["relres"][0] > 1e-10
    # exact solution as the initial guess: converged at the first residual
    Xs, _, _, _, _ = c.orc.pcg(c.Bo, 1e-14)
    B = c.B()
    X0 = dev(Xs)
    o = femcg.default_opts(tol=1e-10, use_x0=1)
    assert femcg.pcg_solve(c.A, B, X0, 1e-10, o) == 0
    assert c.A.stats()["iters"][0] == 0


def test_k_columns_equal_single_solves():
    c = Case(2, 50, 0.3, 1, 4, seed=11)
    rc, X, st = c.solve(1e-12)
    for j in range(c.k):
        B = c.B()[:, j:j + 1].contiguous()
        Xj = torch.zeros_like(B)
        assert femcg.pcg_solve(c.A, B, Xj, 1e-12) == 0
        assert oracle.x_err(Xj.cpu().numpy()[:, 0], X[:, j]) <= 1e-9


def test_batch_equals_alone_bitwise():
    cases = [Case(2, 41, 0.3, 1, 2, seed=21), Case(3, 9, 0.2, 2, 5, seed=22), Case(2, 29, 0.0, 2, 1, seed=23),
             Case(3, 13, 0.3, 1, 8, seed=24)]
    alone = []
    for c in cases:
        rc, X, st = c.solve(1e-10)
        assert rc == 0
        alone.append(X)
    Bs = [c.B() for c in cases]
    Xs = [torch.zeros_like(b) for b in Bs]
    st = femcg.pcg_solve_batch([c.A for c in cases], Bs, Xs, [1e-10] * len(cases))
    torch.cuda.synchronize()
    assert st == [0] * len(cases)
    for X, Xa in zip(Xs, alone):
        assert np.array_equal(X.cpu().numpy(), Xa)


@pytest.mark.parametrize("prec", [femcg.PCG_FP64, femcg.PCG_MIXED])
def test_batch_mixing_one_lane_and_split_rows_bitwise(prec):
    # the kp = 1 class holds one-lane (P1) and split-row (P3, P4) systems, so
    # each SpMM phase launches both kernel instances over the same table
    cases = [Case(2, 80, 0.3, 1, 1, seed=25), Case(2, 25, 0.3, 3, 1, seed=26), Case(2, 20, 0.25, 4, 1, seed=27),
             Case(2, 29, 0.0, 2, 3, seed=28)]
    alone = []
    for c in cases:
        assert c.A.n_free * (4 if c.k == 3 else 1) > 4096  # phase kernels, not the single-workgroup loop
        rc, X, st = c.solve(1e-10, precision=prec)
        assert rc == 0
        assert np.all(c.orc.relres(c.Bo, X) <= 1e-10 * 1.0001)
        alone.append(X)
    Bs = [c.B() for c in cases]
    Xs = [torch.zeros_like(b) for b in Bs]
    st = femcg.pcg_solve_batch([c.A for c in cases], Bs, Xs, [1e-10] * len(cases),
                               femcg.default_opts(tol=1e-10, precision=prec))
    torch.cuda.synchronize()
    assert st == [0] * len(cases)
    for X, Xa in zip(Xs, alone):
        assert np.array_equal(X.cpu().numpy(), Xa)


@pytest.mark.parametrize("order,m", [(3, 23), (4, 17)])
def test_split_rows_mixed_precision_after_tuning(order, m):
    # the tuner's format (CSR or SELL, optional Morton order) with the FP32
    # split-row SpMM inside the refinement loop
    c = Case(2, m, 0.3, order, 1, seed=61, noise=0.01)
    femcg.fem_tune(c.A, 1, femcg.PCG_MIXED)
    Xs, _, _, _, st = c.orc.pcg(c.Bo, 1e-14)
    assert st == 0
    for prec in (femcg.PCG_MIXED, femcg.PCG_FP64):
        rc, X, stats = c.solve(1e-12, precision=prec)
        assert rc == 0, stats
        assert c.orc.relres(c.Bo, X)[0] <= 1e-12 * 1.0001
        assert oracle.x_err(Xs[:, 0], X[:, 0]) <= 1e-8


def test_format_and_tuner_agree():
    c = Case(2, 33, 0.25, 2, 3, seed=31)
    rc, X1, _ = c.solve(1e-12)
    femcg.fem_set_format(c.A, femcg.FEM_FORMAT_CSR)
    rc2, X2, _ = c.solve(1e-12)
    f, cw, sg = femcg.fem_tune(c.A, 3)
    rc3, X3, _ = c.solve(1e-12)
    assert rc == rc2 == rc3 == 0
    assert oracle.x_err(X1, X2) <= 1e-9 and oracle.x_err(X1, X3) <= 1e-9


@pytest.mark.parametrize("dim,m,jit,order,k", [(2, 200, 0.3, 1, 1), (3, 30, 0.2, 1, 8), (2, 60, 0.25, 2, 32),
                                               (3, 12, 0.3, 2, 3), (2, 40, 0.3, 4, 1)])
@pytest.mark.parametrize("prec", [femcg.PCG_FP64, femcg.PCG_MIXED])
def test_band_mode_matches_oracle(dim, m, jit, order, k, prec):
    # band mode with tiny tiles: 145..343 tiles, i.e. several reduction groups
    # of 64 tiles and a ragged last group, folded across blocks in each launch
    c = Case(dim, m, jit, order, k, seed=41, noise=0.01)
    femcg.fem_set_tiling(c.A, 1, 1024)
    Xs, _, _, _, st = c.orc.pcg(c.Bo, 1e-14)
    rc, X, stats = c.solve(1e-12, precision=prec)
    assert rc == 0, stats
    assert np.all(c.orc.relres(c.Bo, X) <= 1e-12 * 1.0001)
    for j in range(c.k):
        assert oracle.x_err(Xs[:, j], X[:, j]) <= 1e-8
    # the SpMM alone, band-mode reduction of p.q exercised by fem_spmv
    rng = np.random.default_rng(5)
    Xr = rng.standard_normal((c.A.n_free, k))
    Y = torch.zeros((c.A.n_free, k), dtype=torch.float64, device="cuda")
    femcg.fem_spmv(c.A, dev(Xr), Y)
    torch.cuda.synchronize()
    Yo = c.orc.spmv(Xr)
    assert np.abs(Y.cpu().numpy() - Yo).max() <= 1e-12 * np.abs(Yo).max()


def test_band_and_tile_modes_agree_and_batch_bitwise():
    cases = [Case(2, 70, 0.3, 1, 2, seed=51), Case(3, 12, 0.2, 1, 4, seed=52)]
    femcg.fem_set_tiling(cases[0].A, 1, 2048)
    femcg.fem_set_tiling(cases[1].A, 0, 0)
    alone = [c.solve(1e-10)[1] for c in cases]
    Bs = [c.B() for c in cases]
    Xs = [torch.zeros_like(b) for b in Bs]
    st = femcg.pcg_solve_batch([c.A for c in cases], Bs, Xs, [1e-10] * 2)
    torch.cuda.synchronize()
    assert st == [0, 0]
    for X, Xa in zip(Xs, alone):
        assert np.array_equal(X.cpu().numpy(), Xa)
    femcg.fem_set_tiling(cases[0].A, 0, 0)
    X0 = cases[0].solve(1e-10)[1]
    assert oracle.x_err(alone[0], X0) <= 1e-7


@pytest.mark.parametrize("dim,m,jit,order,k,fmt,cw", [
    (3, 21, 0.3, 1, 8, femcg.FEM_FORMAT_CSR, 64), (3, 9, 0.2, 2, 3, femcg.FEM_FORMAT_SELL, 32),
    (2, 45, 0.25, 1, 1, femcg.FEM_FORMAT_SELL, 16), (3, 17, 0.0, 1, 32, femcg.FEM_FORMAT_SELL, 64)])
def test_morton_order_matches_oracle(dim, m, jit, order, k, fmt, cw):
    # internal Morton row order: the permutation stays internal, so SpMM and
    # the solve in public DOF order match the oracle exactly as before
    c = Case(dim, m, jit, order, k, seed=61, noise=0.01 if jit else 0.0)
    femcg.fem_set_format(c.A, fmt | femcg.FEM_ORDER_SFC, cw, 1)
    rng = np.random.default_rng(6)
    Xr = rng.standard_normal((c.A.n_free, k))
    Y = torch.zeros((c.A.n_free, k), dtype=torch.float64, device="cuda")
    femcg.fem_spmv(c.A, dev(Xr), Y)
    torch.cuda.synchronize()
    Yo = c.orc.spmv(Xr)
    assert np.abs(Y.cpu().numpy() - Yo).max() <= 1e-12 * np.abs(Yo).max()
    Xs, _, _, _, _ = c.orc.pcg(c.Bo, 1e-14)
    for prec in (femcg.PCG_FP64, femcg.PCG_MIXED):
        rc, X, st = c.solve(1e-12, precision=prec)
        assert rc == 0, st
        assert np.all(c.orc.relres(c.Bo, X) <= 1e-12 * 1.0001)
        for j in range(k):
            assert oracle.x_err(Xs[:, j], X[:, j]) <= 1e-8


def test_tuner_on_3d_and_cold_timing():
    c = Case(3, 19, 0.3, 1, 4, seed=62)
    f, cw, sg = femcg.fem_tune(c.A, 4)
    assert (f & ~femcg.FEM_ORDER_SFC) in (femcg.FEM_FORMAT_CSR, femcg.FEM_FORMAT_SELL)
    rc, X, st = c.solve(1e-10)
    assert rc == 0 and np.all(c.orc.relres(c.Bo, X) <= 1e-10 * 1.0001)
    # the cold-cache probe runs on the copies' own workspaces and leaves the
    # caller's vectors alone
    mats = [c.A] + [femcg.Matrix(c.mesh, 1) for _ in range(3)]
    B = c.B()
    Xt = torch.zeros_like(B)
    ms, by = femcg.pcg_time_spmm_cold(mats, 4, reps=2)
    assert ms > 0 and by > 0
    n, nnz = c.A.n_free, c.A.stats()["nnz_nonzero"]
    assert by >= nnz * 12 + 2 * n * 4 * 8
    rc = femcg.pcg_solve(c.A, B, Xt, 1e-10, femcg.default_opts(tol=1e-10))
    torch.cuda.synchronize()
    assert rc == 0 and np.all(c.orc.relres(c.Bo, Xt.cpu().numpy()) <= 1e-10 * 1.0001)


SMALL_CASES = [(2, 37, 0.3, 1, 1), (2, 23, 0.25, 2, 2), (3, 11, 0.3, 1, 4), (3, 9, 0.3, 2, 1), (2, 64, 0.0, 1, 1),
               (2, 20, 0.3, 1, 8), (2, 10, 0.3, 1, 32), (2, 8, 0.2, 1, 64), (2, 7, 0.3, 3, 2), (2, 6, 0.2, 4, 3)]


@pytest.mark.parametrize("dim,m,jit,order,k", SMALL_CASES)
@pytest.mark.parametrize("prec", [femcg.PCG_FP64, femcg.PCG_MIXED])
def test_single_workgroup_loop_matches_oracle(dim, m, jit, order, k, prec):
    # n * kp <= 4096: the whole loop in one workgroup (mode 2) against the
    # phase kernels (mode 0) and the oracle, (R) at 1e-8 and (S) at 1e-12
    c = Case(dim, m, jit, order, k, seed=71, noise=0.01 if jit else 0.0)
    Xs, _, _, _, st = c.orc.pcg(c.Bo, 1e-14)
    assert st == 0
    _, its_t, _, _, _ = c.orc.pcg(c.Bo, 1e-8)
    res = {}
    for mode in (2, 0):
        femcg.fem_set_tiling(c.A, mode, 0)
        for tol in (1e-8, 1e-12):
            rc, X, stats = c.solve(tol, precision=prec)
            assert rc == 0, (mode, stats)
            assert np.all(c.orc.relres(c.Bo, X) <= tol * 1.0001)
            if tol == 1e-12:
                for j in range(k):
                    assert oracle.x_err(Xs[:, j], X[:, j]) <= 1e-8
                res[mode] = X
            elif prec == femcg.PCG_FP64:
                for j in range(k):
                    assert abs(stats["iters"][j] - its_t[j]) <= 0.02 * its_t[j] + 2, (mode, stats["iters"], its_t)
    for j in range(k):
        assert oracle.x_err(res[0][:, j], res[2][:, j]) <= 1e-9


def test_single_workgroup_mode_limits():
    c = Case(2, 40, 0.3, 1, 4, seed=72)  # n = 1444, kp = 4: above n * kp = 4096
    femcg.fem_set_tiling(c.A, 2, 0)
    with pytest.raises(femcg.FemcgError) as ei:
        c.solve(1e-8)
    assert ei.value.code == femcg.FEMCG_EINVAL
    femcg.fem_set_tiling(c.A, -1, 0)
    rc, X, st = c.solve(1e-10)
    assert rc == 0 and np.all(c.orc.relres(c.Bo, X) <= 1e-10 * 1.0001)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_reentry_after_odd_launch_counts(mode):
    # mixed precision leaves and re-enters the iteration table at every
    # refinement step; with an odd number of iterations per tick the launch
    # index parity changes between entries, and a re-entering system must
    # start from the state slot its residual kernel wrote
    c = Case(2, 30, 0.3, 1, 2, seed=73, noise=0.01)
    femcg.fem_set_tiling(c.A, mode, 0 if mode != 1 else 1024)
    Xs, _, _, _, _ = c.orc.pcg(c.Bo, 1e-14)
    for prec in (femcg.PCG_MIXED, femcg.PCG_FP64):
        for ce in (7, 5, 3):
            rc, X, st = c.solve(1e-12, precision=prec, check_every=ce)
            assert rc == 0, (prec, ce, st)
            assert np.all(c.orc.relres(c.Bo, X) <= 1e-12 * 1.0001)
            for j in range(c.k):
                assert oracle.x_err(Xs[:, j], X[:, j]) <= 1e-8


@pytest.mark.parametrize("dim,m,jit,order", CASES + [(3, 15, 0.3, 2), (2, 70, 0.3, 2)])
def test_device_assembly_equals_host(dim, m, jit, order):
    # same DOFs, same pattern, values to rounding (same summation order; the
    # element arithmetic may contract differently on the two sides)
    mesh = meshgen.make_mesh(dim, m, jit, 17)
    Ah = femcg.Matrix(mesh, order, femcg.FEM_FORMAT_SELL)
    Ad = femcg.Matrix(mesh, order, femcg.FEM_FORMAT_SELL | femcg.FEM_ASSEMBLE_DEVICE)
    for u, v in zip(Ah.dofs(), Ad.dofs()):
        assert np.array_equal(u, v)
    rph, colh, valh = Ah.csr()
    rpd, cold, vald = Ad.csr()
    assert np.array_equal(rph, rpd) and np.array_equal(colh, cold)
    rowmax = np.maximum.reduceat(np.abs(valh), rph[:-1])
    dmax = np.maximum.reduceat(np.abs(vald - valh), rph[:-1])
    assert (dmax / rowmax).max() <= 1e-14
    coords, _, _ = Ah.dofs()
    g = meshgen.harmonic_eval(meshgen.random_coeffs(dim, 3, 4), coords)
    Bh = torch.empty((Ah.n_free, 3), dtype=torch.float64, device="cuda")
    Bd = torch.empty_like(Bh)
    femcg.fem_rhs(Ah, g, Bh)
    femcg.fem_rhs(Ad, g, Bd)
    torch.cuda.synchronize()
    bh, bd = Bh.cpu().numpy(), Bd.cpu().numpy()
    for j in range(3):
        assert np.linalg.norm(bh[:, j] - bd[:, j]) <= 1e-13 * np.linalg.norm(bh[:, j])


def test_device_assembled_solve_matches_oracle():
    c = Case(3, 10, 0.25, 2, 4, seed=19, fmt=femcg.FEM_FORMAT_SELL | femcg.FEM_ASSEMBLE_DEVICE, noise=0.01)
    Xs, _, _, _, _ = c.orc.pcg(c.Bo, 1e-14)
    for prec in (femcg.PCG_FP64, femcg.PCG_MIXED):
        rc, X, st = c.solve(1e-12, precision=prec)
        assert rc == 0
        assert np.all(c.orc.relres(c.Bo, X) <= 1e-12 * 1.0001)
        for j in range(c.k):
            assert oracle.x_err(Xs[:, j], X[:, j]) <= 1e-8
