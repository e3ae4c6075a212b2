"""The library's host assembly (Sect. 2.2's systems, P1-P4) against the oracle
through the C ABI, without a GPU: fem_assemble with FEM_ASSEMBLE_HOST_ONLY
builds the host system and solver copy and allocates no device memory.

Bars as in the GPU assembly parity: DOF coordinates and the Dirichlet /
free-DOF maps bit-equal, identical CSR pattern of A = K_II, and
max_row |dA| / max_row |A| <= 1e-12.  Calls that need the device return
FEMCG_EINVAL on such a matrix and leave it usable.
"""
import numpy as np
import pytest

import meshgen
import oracle
from paper_2201_05413_amd import femcg

CASES = [
    (2, 9, 0.0, 1), (2, 23, 0.3, 1), (3, 6, 0.3, 1),
    (2, 14, 0.25, 2), (3, 5, 0.2, 2), (3, 4, 0.0, 2),
    (2, 11, 0.3, 3), (2, 9, 0.25, 4), (2, 3, 0.0, 4),
]


def _host_matrix(mesh, order, fmt=femcg.FEM_FORMAT_SELL):
    return femcg.Matrix(mesh, order, fmt | femcg.FEM_ASSEMBLE_HOST_ONLY)


@pytest.mark.parametrize("dim,m,jit,order", CASES)
def test_host_assembly_matches_oracle(dim, m, jit, order):
    mesh = meshgen.make_mesh(dim, m, jit, 7)
    A = _host_matrix(mesh, order)
    orc = oracle.System(mesh, order)
    coords_l, dir_l, f2d_l = A.dofs()
    coords_o, dir_o, f2d_o = orc.dofs()
    assert np.array_equal(coords_l, coords_o)
    assert np.array_equal(dir_l, dir_o) and np.array_equal(f2d_l, f2d_o)
    rp, col, val = A.csr()
    rpo, colo, valo = orc.A()
    assert np.array_equal(rp, rpo) and np.array_equal(col, colo)
    rowmax = np.maximum.reduceat(np.abs(valo), rpo[:-1])
    dmax = np.maximum.reduceat(np.abs(val - valo), rpo[:-1])
    assert (dmax / rowmax).max() <= 1e-12
    st = A.stats()
    assert st["n"] == orc.nfree and st["nnz"] == len(valo)


@pytest.mark.parametrize("fmt", [femcg.FEM_FORMAT_CSR, femcg.FEM_FORMAT_SELL])
def test_host_assembly_is_independent_of_the_solver_format(fmt):
    mesh = meshgen.make_mesh(2, 15, 0.3, 2)
    a = _host_matrix(mesh, 2, fmt).csr()
    b = _host_matrix(mesh, 2, femcg.FEM_FORMAT_SELL | femcg.FEM_ORDER_SFC).csr()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)  # the public CSR is in public row order


def test_device_calls_are_rejected_on_a_host_only_matrix():
    mesh = meshgen.make_mesh(2, 8, 0.2, 3)
    A = _host_matrix(mesh, 1)
    n = A.n_free
    host = np.zeros((n, 1))
    lib = femcg.lib()
    P = femcg.C.c_void_p
    p = P(host.ctypes.data)
    g = np.zeros((A.n_all, 1))
    calls = [lambda: lib.fem_rhs(A.h, P(g.ctypes.data), 1, p, None),
             lambda: lib.fem_spmv(A.h, p, p, 1, None),
             lambda: lib.pcg_solve(A.h, p, p, 1, 1e-8, None, None),
             lambda: lib.fem_set_format(A.h, femcg.FEM_FORMAT_CSR, 64, 1),
             lambda: lib.fem_tune(A.h, 1, femcg.PCG_FP64, None, None, None),
             lambda: lib.bicgstab_solve(A.h, p, p, 1e-8, 4, None, 0, None, None)]
    for call in calls:
        assert call() == femcg.FEMCG_EINVAL
        assert b"FEM_ASSEMBLE_HOST_ONLY" in lib.fem_last_error()
    # still usable afterwards
    rp, col, val = A.csr()
    assert rp[-1] == len(val) > 0


def test_device_and_host_only_flags_exclude_each_other():
    mesh = meshgen.make_mesh(2, 6, 0.0, 1)
    with pytest.raises(femcg.FemcgError) as ei:
        femcg.Matrix(mesh, 1, femcg.FEM_FORMAT_SELL | femcg.FEM_ASSEMBLE_DEVICE | femcg.FEM_ASSEMBLE_HOST_ONLY)
    assert ei.value.code == femcg.FEMCG_EINVAL


def test_binding_checks_bicgstab_arguments_before_any_device_call():
    torch = pytest.importorskip("torch")
    A = _host_matrix(meshgen.make_mesh(2, 8, 0.2, 3), 1)
    B = torch.zeros(A.n_free, dtype=torch.float64)
    with pytest.raises(ValueError):
        femcg.bicgstab_solve(A, B, B, 1e-8, 4, row_scale=np.ones(A.n_free + 1))
    with pytest.raises(ValueError):
        femcg.bicgstab_solve(A, torch.zeros(A.n_free + 1, dtype=torch.float64), B, 1e-8, 4)
    with pytest.raises(TypeError):  # host tensors: the boundary takes device memory
        femcg.bicgstab_solve(A, B, B, 1e-8, 4, row_scale=np.ones(A.n_free))
