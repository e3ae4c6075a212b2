"""The continuous-batching server through the C ABI: every request's solution
is bit-identical to the same system solved alone (batch invariance of the
phase and single-workgroup kernels) and passes the oracle's Eq. (2) check."""
import ctypes as C

import numpy as np
import pytest

import meshgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2201_05413_amd import femcg  # noqa: E402

# (dim, m, jitter, order, k): single-workgroup, tile-mode P2 3D (assembled on
# the device), tile-mode P1, P2 2D with two columns, P3 with two columns, and
# P4 with one column (split-row SpMM beside the one-lane P1 in one kp class)
REQS = [(2, 30, 0.3, 1, 3), (3, 14, 0.2, 2, 5), (2, 90, 0.3, 1, 1), (2, 50, 0.0, 2, 2), (2, 25, 0.3, 3, 2),
        (2, 18, 0.25, 4, 1)]


def _request(i, dim, m, jit, order, k):
    mesh = meshgen.make_mesh(dim, m, jit, 80 + i)
    orc = oracle.System(mesh, order)
    coords, _, _ = orc.dofs()
    g = np.ascontiguousarray(meshgen.harmonic_eval(meshgen.random_coeffs(dim, k, 90 + i), coords))
    return mesh, orc, g


@pytest.mark.parametrize("prec", [femcg.PCG_FP64, femcg.PCG_MIXED])
def test_server_results_equal_solo_solves(prec):
    tol, ce = 1e-9, 16
    reqs = [_request(i, *r) for i, r in enumerate(REQS)]
    L = femcg.lib()
    srv = C.c_void_p()
    femcg._check(L.serve_create(8e9, 8, prec, ce, C.byref(srv)))
    try:
        ids, keep = [], []
        for (dim, m, jit, order, k), (mesh, _, g) in zip(REQS, reqs):
            ms, hold = femcg.make_mesh_struct(mesh)
            keep.append(hold)
            rid = L.serve_submit(srv, C.byref(ms), order, femcg._np_ptr(g), k, tol)
            femcg._check(rid)
            ids.append(rid)
        for _ in range(100000):
            left = L.serve_step(srv)
            femcg._check(left)
            if left == 0:
                break
        assert left == 0
        got = []
        for (dim, m, jit, order, k), (mesh, orc, g), rid in zip(REQS, reqs, ids):
            n = orc.nfree
            X = np.zeros((n, k))
            info = femcg.fem_request_info()
            assert L.serve_poll(srv, rid, femcg._np_ptr(X), C.byref(info)) == 1
            assert info.status == 0
            got.append(X)
    finally:
        L.serve_destroy(srv)
    for (dim, m, jit, order, k), (mesh, orc, g), X in zip(REQS, reqs, got):
        # (R): the oracle's own residual of the served solution
        Bo = orc.rhs(g)
        assert np.all(orc.relres(Bo, X) <= tol * 1.0001)
        # the same system alone, assembled where the server assembles it
        # (on the device from 2^20 element entries on): bit-identical
        nvl = dim + 1
        nl = nvl if order == 1 else (nvl + nvl * (nvl - 1) // 2 if order == 2 else (order + 1) * (order + 2) // 2)
        big = mesh["cells"].shape[0] * nl * nl >= 1 << 20
        A = femcg.Matrix(mesh, order, femcg.FEM_FORMAT_SELL | (femcg.FEM_ASSEMBLE_DEVICE if big else 0))
        B = torch.empty((A.n_free, k), dtype=torch.float64, device="cuda")
        femcg.fem_rhs(A, g, B)
        Xs = torch.zeros_like(B)
        assert femcg.pcg_solve(A, B, Xs, tol, femcg.default_opts(tol=tol, precision=prec, check_every=ce)) == 0
        torch.cuda.synchronize()
        assert np.array_equal(Xs.cpu().numpy(), X)
