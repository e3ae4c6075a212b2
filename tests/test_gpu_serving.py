"""The continuous-batching server through the C ABI: every request's solution
is bit-identical to the same system solved alone (batch invariance of the
phase and single-workgroup kernels) and passes the oracle's Eq. (2) check."""
import ctypes as C
import time

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


# requests for the pressure test: 2D P1, 3D P1, P2 and P3 systems with k in
# 9..16, so every request runs the kp = 16 phase kernels and the footprints
# (dominated by the per-tile partials of kp = 16) are close: any two fit the
# budget and no three do.  (2, 300, ...) is larger than the whole budget.
PRESSURE = [(2, 40, 0.3, 1, 12), (3, 12, 0.2, 1, 16), (2, 22, 0.0, 2, 10), (2, 38, 0.3, 1, 16), (2, 16, 0.3, 3, 9)]
TOO_BIG = (2, 300, 0.3, 1, 16)


def _drain(L, srv, ids, out, X_of):
    """Poll every id in `ids`; store (info, X) of the finished ones in out."""
    for rid in list(ids):
        i = ids[rid]
        X = X_of(i)
        info = femcg.fem_request_info()
        if L.serve_poll(srv, rid, femcg._np_ptr(X) if X is not None else None, C.byref(info)) == 1:
            out[i] = (info, X)
            del ids[rid]


@pytest.mark.parametrize("prec", [femcg.PCG_FP64, femcg.PCG_MIXED])
def test_server_under_memory_pressure(prec):
    # Continuous batching under pressure: a budget that holds about two
    # requests and two slots; requests arrive between ticks while others run,
    # queue until a retirement frees memory, and one request larger than the
    # budget is rejected with FEMCG_EADMIT.  Every served result equals the
    # solo solve bit for bit and passes the oracle's Eq. (2) check.
    tol, ce = 1e-9, 8
    L = femcg.lib()
    reqs = [_request(20 + i, *r) for i, r in enumerate(PRESSURE)]
    big = _request(40, *TOO_BIG)
    keep = []

    def submit(srv, mesh, order, g, k):
        ms, hold = femcg.make_mesh_struct(mesh)
        keep.append(hold)
        rid = L.serve_submit(srv, C.byref(ms), order, femcg._np_ptr(g), k, tol)
        femcg._check(rid)
        return rid

    # footprints as the server counts them, from a roomy probe server
    srv = C.c_void_p()
    femcg._check(L.serve_create(8e9, 8, prec, ce, C.byref(srv)))
    try:
        ids = {submit(srv, mesh, r[3], g, r[4]): i for i, (r, (mesh, _, g)) in enumerate(zip(PRESSURE, reqs))}
        while L.serve_step(srv) > 0:
            pass
        probe = {}
        _drain(L, srv, ids, probe, lambda i: None)
    finally:
        L.serve_destroy(srv)
    fp = sorted(probe[i][0].footprint_mb * 1e6 for i in range(len(PRESSURE)))
    assert fp[0] > 0
    # any two requests fit the budget and no three do: memory, not the slot
    # count, is what makes later arrivals wait
    budget = 1.01 * (fp[-1] + fp[-2])
    assert fp[0] + fp[1] + fp[2] > budget
    srv = C.c_void_p()
    femcg._check(L.serve_create(budget, 4, prec, ce, C.byref(srv)))
    got = {}
    try:
        ids = {}
        nxt = 0
        big_id = None
        # tick -> submissions before it; the first two need more than two
        # ticks of check_every iterations, so the third arrives while they run
        schedule = {0: 2, 2: 1, 3: "big", 5: 2}
        for tick in range(100000):
            sub = schedule.get(tick, 0)
            if sub == "big":
                big_id = submit(srv, big[0], TOO_BIG[3], big[2], TOO_BIG[4])
            else:
                for _ in range(sub):
                    r = PRESSURE[nxt]
                    ids[submit(srv, reqs[nxt][0], r[3], reqs[nxt][2], r[4])] = nxt
                    nxt += 1
            if sub:
                time.sleep(0.5)  # host assembly runs on the server's own thread
            left = L.serve_step(srv)
            femcg._check(left)
            _drain(L, srv, ids, got, lambda i: np.zeros((reqs[i][1].nfree, PRESSURE[i][4])))
            if left == 0 and tick > max(schedule):
                break
        assert nxt == len(PRESSURE) and not ids
        info = femcg.fem_request_info()
        assert L.serve_poll(srv, big_id, None, C.byref(info)) == 1
        assert info.status == femcg.FEMCG_EADMIT and info.footprint_mb * 1e6 > budget
    finally:
        L.serve_destroy(srv)
    infos = [got[i][0] for i in range(len(PRESSURE))]
    for i, inf in enumerate(infos):
        assert inf.status == 0, (i, inf.status)
        assert inf.footprint_mb == probe[i][0].footprint_mb
    # queueing happened: some request was admitted only after another retired
    assert any(a.t_admit >= b.t_done for a in infos for b in infos if a is not b)
    # and requests overlapped on the device
    assert any(a.t_admit < b.t_done and b.t_admit < a.t_done for a in infos for b in infos if a is not b)
    for i, ((dim, m, jit, order, k), (mesh, orc, g)) in enumerate(zip(PRESSURE, reqs)):
        X = got[i][1]
        assert np.all(orc.relres(orc.rhs(g), X) <= tol * 1.0001), i
        A = femcg.Matrix(mesh, order, femcg.FEM_FORMAT_SELL)
        B = torch.empty((A.n_free, k), dtype=torch.float64, device="cuda")
        femcg.fem_rhs(A, g, B)
        Xs = torch.zeros_like(B)
        assert femcg.pcg_solve(A, B, Xs, tol, femcg.default_opts(tol=tol, precision=prec, check_every=ce)) == 0
        torch.cuda.synchronize()
        assert np.array_equal(Xs.cpu().numpy(), X), i


def test_device_assembly_beside_running_solves():
    # small requests start solving at once while the larger ones are still
    # being assembled on the device by the server's worker threads; every
    # served solution must pass the oracle's own Eq. (2) check
    small = [(2, 40 + 3 * i, 0.3 * (i % 2), 1 + (i % 2), 1 + (i % 5)) for i in range(12)]
    big = [(3, 28, 0.0, 1, 2), (2, 180, 0.3, 2, 3), (3, 14, 0.2, 2, 4), (2, 200, 0.0, 2, 2)]
    spec = small[:6] + big[:2] + small[6:] + big[2:]
    for dim, m, jit, order, k in big:
        nvl = dim + 1
        nl = nvl if order == 1 else nvl + nvl * (nvl - 1) // 2
        cells = (m - 1) ** dim * (2 if dim == 2 else 6)
        assert cells * nl * nl >= 1 << 20  # assembled on the device by the server
    tol = 1e-8
    reqs = [_request(100 + i, *r) for i, r in enumerate(spec)]
    L = femcg.lib()
    srv = C.c_void_p()
    femcg._check(L.serve_create(16e9, 16, femcg.PCG_FP64, 16, C.byref(srv)))
    try:
        ids, keep = [], []
        for (dim, m, jit, order, k), (mesh, _, g) in zip(spec, reqs):
            ms, hold = femcg.make_mesh_struct(mesh)
            keep.append(hold)
            rid = L.serve_submit(srv, C.byref(ms), order, femcg._np_ptr(g), k, tol)
            femcg._check(rid)
            ids.append(rid)
            femcg._check(L.serve_step(srv))  # the engine runs while later requests assemble
        for _ in range(100000):
            left = L.serve_step(srv)
            femcg._check(left)
            if left == 0:
                break
        assert left == 0
        got = []
        for (dim, m, jit, order, k), (mesh, orc, g), rid in zip(spec, reqs, ids):
            X = np.zeros((orc.nfree, k))
            info = femcg.fem_request_info()
            assert L.serve_poll(srv, rid, femcg._np_ptr(X), C.byref(info)) == 1
            assert info.status == 0
            got.append(X)
    finally:
        L.serve_destroy(srv)
    for (dim, m, jit, order, k), (mesh, orc, g), X in zip(spec, reqs, got):
        assert np.all(orc.relres(orc.rhs(g), X) <= tol * 1.0001), (dim, m, jit, order, k)
