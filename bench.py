"""Benchmark of the Jacobi-PCG hot path on one MI355X.

One step = one full pass of the path over the workload's system, inputs
resident in HBM: lift the Dirichlet data into B on the device, solve to the
tolerance with plain FP64 PCG, then solve again with the FP32-inner /
FP64-refined PCG (iterations as HIP graph replays, alpha/beta/convergence on
the device).  Reported: whole-step algorithmic GB/s (value), time-to-tol of
both precisions and their ratio, p50/p99 of the per-solve latency over the
timed steps, the roofline of the dominant kernel (SpMM + p.q of the FP64
iteration, timed with HIP events on its stream), and the oracle on the host
CPU as a bounded-sample baseline.

Default workload: 3D P1 on the structured 128^3 vertex cube, 6 Kuhn
tetrahedra per cell (2,000,376 unknowns), 32 right-hand sides of random
harmonic cubic Dirichlet data, tol 1e-8: the largest single-GPU solve
configuration, whose iteration working set (1.2 GB per SpMM) streams from
HBM.  Other workloads: --workload c1|c2|c4 (single solves; c2's working set
sits in the 256 MB Infinity Cache), c5 (serving stream),
asm (host vs device assembly), deg (P1..P4 on one mesh, as in Table 7),
bcg (the paper's BiCGStab + Block-Jacobi against Jacobi-PCG), rhs (the
iterative side of Sect. 4.3's multiple right-hand-side model).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpMV HBM GB/s + time-to-1e-8 residual vs FP64 PCG; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    i = min(len(xs) - 1, max(0, int(math.ceil(p / 100.0 * len(xs))) - 1))
    return xs[i]


def iter_bytes(n, nnz, k, sv):
    """Algorithmic HBM bytes of one fused PCG iteration."""
    return nnz * (sv + 4) + 4 * (n + 1) + 10 * n * k * sv + 2 * n * sv


def pad_k(k):
    """Lanes per row: the column count padded to a power of two."""
    kp = 1
    while kp < k:
        kp *= 2
    return kp


def spmm_bytes(n, nnz, k, sv):
    return nnz * (sv + 4) + 4 * n + 2 * n * k * sv


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, orc, g, nnz_kept, gpu_iters, budget_s=20.0):
    """The oracle on the host CPU, on a bounded sample of the same solve.

    Two timings of the oracle's Jacobi-PCG (plain C, FP64): the default
    one-thread build on column 0, and the all-core build (the same loops
    built with -fopenmp; the k columns run on separate threads, each with
    the one-thread arithmetic) on every column.  Each runs a capped number
    of iterations sized to about budget_s / 2 seconds; time-to-tol is that
    rate times the GPU FP64 solve's iteration count.  Rates use the GPU
    line's algorithmic bytes (kept nonzeros)."""
    import numpy as np
    import oracle

    B = orc.rhs(g)
    n, k = B.shape
    rp, col, val = orc.A()
    its_tol = int(max(gpu_iters))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
    # one thread, column 0
    t0 = time.time()
    oracle.pcg_csr(rp, col, val, B[:, :1], 1e-300, max_iter=3)
    dt = max(time.time() - t0, 1e-3) / 3
    cap1 = max(5, min(its_tol, int(0.5 * budget_s / dt)))
    t0 = time.time()
    _, it1, _, _, _ = oracle.pcg_csr(rp, col, val, B[:, :1], 1e-300, max_iter=cap1)
    el1 = time.time() - t0
    ms1 = 1e3 * el1 / int(it1[0])
    # all cores, every column
    t0 = time.time()
    oracle.pcg_csr(rp, col, val, B, 1e-300, max_iter=3, threads=threads)
    dtk = max(time.time() - t0, 1e-3) / 3
    capk = max(5, min(its_tol, int(0.5 * budget_s / dtk)))
    t0 = time.time()
    _, itk, _, _, _ = oracle.pcg_csr(rp, col, val, B, 1e-300, max_iter=capk, threads=threads)
    elk = time.time() - t0
    assert int(itk.min()) == capk
    msk = 1e3 * elk / capk  # all k columns advance one iteration
    used = min(threads, k)
    rate = iter_bytes(n, nnz_kept, k, 8) * capk / elk / 1e9
    return dict(value=round(rate, 3), unit="GB/s", cores=used, kind="oracle", cpu_model=cpu_model(),
                host_threads=os.cpu_count(),
                time_to_tol_s=round(msk * its_tol / 1e3, 2), time_to_tol_kind="extrapolated",
                iters_to_tol=its_tol,
                sample="oracle FP64 Jacobi-PCG, all-core build (-fopenmp, %d threads, one column per thread "
                       "at a time): the %d columns of %s for %d iterations (%.1f s, %.1f ms per iteration of "
                       "all columns); time_to_tol_s = that rate x %d iterations (GPU FP64 count)"
                       % (used, k, w.name, capk, elk, msk, its_tol),
                single_thread={"value": round(iter_bytes(n, nnz_kept, 1, 8) * int(it1[0]) / el1 / 1e9, 3),
                               "unit": "GB/s", "cores": 1, "ms_per_iter_per_column": round(ms1, 2),
                               "time_to_tol_s": round(ms1 * its_tol * k / 1e3, 2),
                               "sample": "column 0, %d iterations (%.1f s); time-to-tol = %d columns x %d "
                                         "iterations at that rate" % (int(it1[0]), el1, k, its_tol)})


def calibration_copy(args):
    """One plain device copy of --calibrate-copy-mb (HBM counter calibration)."""
    import torch

    if args.calibrate_copy_mb > 0:
        nel = int(args.calibrate_copy_mb * 1e6 / 8)
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d doubles (%.1f MB read, %.1f MB written)" % (nel, nel * 8e-6, nel * 8e-6))
        del src, dst


def make_workload(name):
    import meshgen
    return {"c1": meshgen.c1, "c2": meshgen.c2, "c3": meshgen.c3, "c4": meshgen.c4}[name]()


def run_single(args):
    import numpy as np
    import torch

    import oracle
    from paper_2201_05413_amd import femcg

    torch.cuda.set_device(0)
    calibration_copy(args)
    t0 = time.time()
    w = make_workload(args.workload)
    log("workload %s: mesh %.1f s" % (w.name, time.time() - t0))
    t0 = time.time()
    A = femcg.Matrix(w.mesh, w.order, femcg.FEM_FORMAT_SELL)
    t_asm = time.time() - t0
    coords, _, f2d = A.dofs()
    g = w.dirichlet(coords)
    k = w.k
    n = A.n_free
    B = torch.empty((n, k), dtype=torch.float64, device="cuda")
    X64 = torch.zeros_like(B)
    Xmx = torch.zeros_like(B)
    femcg.fem_rhs(A, g, B)
    t0 = time.time()
    order = 0
    tune = None
    eta = args.eta
    if args.format == "auto":
        # the whole solve tuned on this workload's B: format and row order,
        # lanes per row, tiling, precision and inner tolerance
        _, tune = femcg.pcg_tune(A, B, w.tol, femcg.default_opts(tol=w.tol, check_every=args.check_every))
        fmt, cw, sg = tune["format"], tune["C"], tune["sigma"]
        order = femcg.FEM_ORDER_SFC if tune["sfc"] else 0
        if tune["inner_eta"] > 0:
            eta = tune["inner_eta"]
    else:
        parts = args.format.split(":")
        fmt = femcg.FEM_FORMAT_CSR if parts[0] == "csr" else femcg.FEM_FORMAT_SELL
        cw = int(parts[1]) if len(parts) > 1 else 64
        sg = int(parts[2]) if len(parts) > 2 else 1
        order = femcg.FEM_ORDER_SFC if args.order == "sfc" else 0
        femcg.fem_set_format(A, fmt | order, cw, sg)
    if args.band is not None:
        femcg.fem_set_tiling(A, args.band, args.tile)
    t_tune = time.time() - t0
    log("assembly %.2f s, tuner %.2f s -> format %d C=%d sigma=%d order %s" % (t_asm, t_tune, fmt, cw, sg,
                                                                               "sfc" if order else "natural"))
    o64 = femcg.default_opts(tol=w.tol, precision=femcg.PCG_FP64, check_every=args.check_every)
    omx = femcg.default_opts(tol=w.tol, precision=femcg.PCG_MIXED, check_every=args.check_every,
                             inner_eta=eta)
    stream = torch.cuda.current_stream()

    def step():
        ta = time.perf_counter()
        femcg.fem_rhs(A, g, B)
        rc1 = femcg.pcg_solve(A, B, X64, w.tol, o64)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        s64 = A.stats()
        rc2 = femcg.pcg_solve(A, B, Xmx, w.tol, omx)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        smx = A.stats()
        if rc1 != 0 or rc2 != 0:
            raise RuntimeError("solve status %d / %d" % (rc1, rc2))
        return tb - ta, tc - tb, s64, smx

    if args.profile:
        # short run for hardware-counter passes: a capped FP64 solve, then
        # the three iteration kernels timed on its workspace
        femcg.pcg_solve(A, B, X64, w.tol, femcg.default_opts(tol=w.tol, max_iter=args.profile,
                                                              check_every=args.check_every))
        torch.cuda.synchronize()
        for kk in range(3):
            ms, by = femcg.pcg_time_kernel(A, kk, reps=args.kernel_reps)
            log("kernel %d: %.4f ms, %.1f GB/s" % (kk, ms, by / ms / 1e6))
        return
    for i in range(args.warmup):
        step()
        log("warmup %d done" % i)
    torch.cuda.synchronize()
    lat64, latmx, bytes_tot = [], [], 0.0
    T0 = time.perf_counter()
    for i in range(args.steps):
        t64, tmx, s64, smx = step()
        lat64.append(t64)
        latmx.append(tmx)
        bytes_tot += s64["bytes"] + smx["bytes"]
        log("step %d: fp64 %.2f ms (%d its), mixed %.2f ms (%d inner its, %d outer)"
            % (i, 1e3 * t64, max(s64["iters"]), 1e3 * tmx, max(smx["iters"]), smx["outer"]))
    torch.cuda.synchronize()
    T = time.perf_counter() - T0
    # parity (R): the oracle's own residual of both solutions
    x64 = X64.cpu().numpy()
    xmx = Xmx.cpu().numpy()
    diff = float(np.linalg.norm(xmx - x64) / np.linalg.norm(x64))
    rel64 = relmx = np.array([float("nan")])
    orc = None
    if not args.no_check or not args.no_cpu:
        t0 = time.time()
        orc = oracle.System(w.mesh, w.order)
        log("oracle assembly %.1f s" % (time.time() - t0))
    if not args.no_check:
        t0 = time.time()
        Bo = orc.rhs(g)
        rel64 = orc.relres(Bo, x64)
        relmx = orc.relres(Bo, xmx)
        log("oracle check %.1f s: relres fp64 %.3e mixed %.3e (tol %.0e)" % (time.time() - t0, rel64.max(),
                                                                             relmx.max(), w.tol))
    # Eq. (1) error against the exact discrete solution, where the data make
    # it known in closed form: the nodal values of g (linear data on P1,
    # harmonic cubics on the structured Kuhn cube, x^2 - y^2 on P2)
    exact_cols = {"c1": range(k), "c3": range(k), "c4": [0]}.get(args.workload, [])
    xerr = None
    if exact_cols:
        gf = g.reshape(g.shape[0], -1)[f2d]
        xerr = {"columns": len(exact_cols),
                "fp64_max": max(oracle.x_err(gf[:, j], x64[:, j]) for j in exact_cols),
                "mixed_max": max(oracle.x_err(gf[:, j], xmx[:, j]) for j in exact_cols),
                "reference": "nodal values of the Dirichlet data (the exact discrete solution)"}
    # roofline of the dominant kernel: SpMM + p.q of the FP64 iteration
    femcg.pcg_solve(A, B, X64, w.tol, o64)
    torch.cuda.synchronize()
    st = A.stats()
    ms_spmm, by_spmm = femcg.pcg_time_kernel(A, 0, reps=args.kernel_reps)
    ms_upd, by_upd = femcg.pcg_time_kernel(A, 1, reps=args.kernel_reps)
    ms_pup, by_pup = femcg.pcg_time_kernel(A, 2, reps=args.kernel_reps)
    # restore the solution overwritten by the forced kernel launches
    femcg.pcg_solve(A, B, X64, w.tol, o64)
    torch.cuda.synchronize()
    achieved = by_spmm / (ms_spmm * 1e-3) / 1e9
    cold = None
    # (a system whose SpMM moves under 16 MB is latency-bound: no cold rate)
    if args.cold_mb > 0 and by_spmm >= 16e6:
        # the same SpMM on rotating copies whose total far exceeds the 256 MB
        # last-level cache: no launch finds its operands cache-resident
        ncopy = min(128, max(4, int(math.ceil(args.cold_mb * 1e6 / by_spmm))))
        t0 = time.time()
        mats = [A]
        for _ in range(ncopy - 1):
            Ac = femcg.Matrix(w.mesh, w.order, femcg.FEM_FORMAT_SELL)
            femcg.fem_set_format(Ac, fmt | order, cw, sg)
            if args.band is not None:
                femcg.fem_set_tiling(Ac, args.band, args.tile)
            elif tune is not None and tune["band"] in (0, 1):
                femcg.fem_set_tiling(Ac, tune["band"], tune["tile"])
            mats.append(Ac)
        ms_c, by_c = femcg.pcg_time_spmm_cold(mats, k, femcg.PCG_FP64, reps=5)
        cold = {"copies": ncopy, "aggregate_mb": round(ncopy * by_c / 1e6, 1), "ms": round(ms_c, 5),
                "gbs": round(by_c / (ms_c * 1e-3) / 1e9, 1),
                "frac": round(by_c / (ms_c * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log("cold-cache SpMM over %d copies (%.0f MB, set-up %.1f s): %.4f ms, %.1f GB/s"
            % (ncopy, ncopy * by_c / 1e6, time.time() - t0, ms_c, cold["gbs"]))
        for Ac in mats[1:]:
            Ac.free()
        del mats
        # the copies' probes overwrote only their own workspaces, but the
        # first matrix's p was zero-filled: restore its solution state
        femcg.pcg_solve(A, B, X64, w.tol, o64)
        torch.cuda.synchronize()
    traffic = None
    if args.traffic_json and os.path.exists(args.traffic_json):
        traffic = json.load(open(args.traffic_json)).get(w.name)
    # one iteration's working set (matrix, x, r, p, q, D^-1) against the
    # 256 MB last-level (Infinity) cache: beyond it the SpMM streams from HBM
    sv = 8
    work_set = st["nnz_nonzero"] * (sv + 4) + 4 * n * pad_k(k) * sv + n * sv
    bound = "hbm" if work_set > 256e6 else "cache"
    line = {
        "metric": METRIC,
        "value": round(bytes_tot / T / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * T / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (FP64 PCG) + f32-inner/f64-refined (mixed PCG)",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "recipe": meshgen_doc(args.workload),
            "n": n, "nnz_structural": st["nnz"], "nnz_nonzero": st["nnz_nonzero"], "k": k, "tol": w.tol,
            "format": {0: "CSR", 1: "SELL"}[fmt], "sell_C": cw, "sell_sigma": sg,
            "row_order": "morton" if order else "natural",
        },
        "time_to_tol_ms": {"fp64_p50": round(1e3 * percentile(lat64, 50), 3),
                           "mixed_p50": round(1e3 * percentile(latmx, 50), 3),
                           "mixed_over_fp64": round(percentile(latmx, 50) / percentile(lat64, 50), 3),
                           "mixed_inner_eta": eta,
                           "tuned_choice": None if tune is None else ("fp64" if tune["fp64_fallback"] else "mixed"),
                           "tuned_p50": round(1e3 * min(percentile(lat64, 50), percentile(latmx, 50))
                                              if tune is None or not tune["fp64_fallback"]
                                              else 1e3 * percentile(lat64, 50), 3)},
        "tuner": tune,
        "latency_ms": {"fp64_p50": round(1e3 * percentile(lat64, 50), 3),
                       "fp64_p99": round(1e3 * percentile(lat64, 99), 3),
                       "mixed_p50": round(1e3 * percentile(latmx, 50), 3),
                       "mixed_p99": round(1e3 * percentile(latmx, 99), 3)},
        "iters": {"fp64": st["iters"], "mixed_inner_last": None},
        "parity": {"oracle_relres_fp64": float(rel64.max()), "oracle_relres_mixed": float(relmx.max()),
                   "mixed_vs_fp64_rel_l2": diff, "x_err_vs_exact": xerr},
        "spmm_cold_rotated": cold,
        "kernels_ms": {"spmm_pq": round(ms_spmm, 5), "update": round(ms_upd, 5), "pupdate": round(ms_pup, 5)},
        "kernels_gbs": {"spmm_pq": round(achieved, 1), "update": round(by_upd / (ms_upd * 1e-3) / 1e9, 1),
                        "pupdate": round(by_pup / (ms_pup * 1e-3) / 1e9, 1)},
        "roofline": {"bound": bound, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_spmm<double,%d> (SpMM + p.q, FP64)" % pad_k(k), "bytes_per_launch": by_spmm,
                     "iteration_working_set_mb": round(work_set / 1e6, 1),
                     "note": ("working set beyond the 256 MB Infinity Cache: HBM-bound" if bound == "hbm" else
                              "working set inside the 256 MB Infinity Cache: cache-resident, not an HBM "
                              "figure (see spmm_cold_rotated for the HBM rate)")},
    }
    if not args.no_cpu:
        t0 = time.time()
        line["cpu_baseline"] = cpu_baseline(w, orc, g, st["nnz_nonzero"], st["iters"], args.cpu_budget)
        log("cpu baseline %.1f s" % (time.time() - t0))
    print(json.dumps(line), flush=True)


def run_serve(args):
    """Serving stream: Poisson arrivals of mixed 2D/3D, P1/P2, structured/jittered
    requests with 1..16 random harmonic right-hand sides, tol 1e-8.  First the
    server's capacity (every request submitted at once), then the same requests
    replayed as Poisson arrivals at fractions of that capacity (0.5x and 1x by
    default); one-at-a-time FP64 PCG replays the trace nearest 0.7x capacity
    for comparison."""
    import ctypes as C

    import numpy as np
    import torch

    import meshgen
    from paper_2201_05413_amd import femcg

    torch.cuda.set_device(0)
    # arrival times at rate 1; a trace at rate r divides them by r
    reqs = meshgen.request_stream(args.n_requests, 1.0, seed=6, max2d=args.max2d, max3d=args.max3d)
    t0 = time.time()
    wls = []
    for r in reqs:
        wls.append(meshgen.build_request(r))
        if len(wls) % 50 == 0:
            log("generated %d of %d requests" % (len(wls), len(reqs)))
    log("generated %d requests in %.1f s" % (len(wls), time.time() - t0))
    # DOF coordinates (public order) of every request, for its Dirichlet data:
    # P1 = vertices; P2 = vertices then edge midpoints in (min, max) order
    gs = []
    for w in wls:
        coords = w.mesh["coords"]
        if w.order == 2:
            cells = w.mesh["cells"]
            d = cells.shape[1]
            pairs = []
            for a in range(d):
                for b in range(a + 1, d):
                    lo = np.minimum(cells[:, a], cells[:, b]).astype(np.int64)
                    hi = np.maximum(cells[:, a], cells[:, b]).astype(np.int64)
                    pairs.append(lo * (1 << 32) + hi)
            e = np.unique(np.concatenate(pairs))
            mid = 0.5 * (coords[e >> 32] + coords[e & 0xFFFFFFFF])
            coords = np.concatenate([coords, mid])
        gs.append(np.ascontiguousarray(w.dirichlet(coords)))
    prec = femcg.PCG_MIXED if args.serve_mixed else femcg.PCG_FP64
    L = femcg.lib()
    meshes = [femcg.make_mesh_struct(w.mesh) for w in wls]
    # free-DOF maps from the library's host-only assembly (no device memory)
    f2ds = []
    for w in wls:
        H = femcg.Matrix(w.mesh, w.order, femcg.FEM_FORMAT_CSR | femcg.FEM_ASSEMBLE_HOST_ONLY)
        f2ds.append(H.dofs()[2])
        H.free()
    nfree = [len(f) for f in f2ds]
    xs, done_cap = {}, {}

    def serve(t_arr, keep_x=False, what=""):
        """Replay arrival times t_arr (seconds) through a fresh server; with
        keep_x, return every served solution as well."""
        srv = C.c_void_p()
        femcg._check(L.serve_create(args.budget_gb * 1e9, args.slots, prec, args.check_every, C.byref(srv)))
        ids, done = {}, {}
        t_start = L.serve_clock(srv)
        nxt = 0
        while len(done) < len(wls):
            now = L.serve_clock(srv) - t_start
            while nxt < len(wls) and t_arr[nxt] <= now:
                m, _ = meshes[nxt]
                rid = L.serve_submit(srv, C.byref(m), wls[nxt].order, femcg._np_ptr(gs[nxt]), wls[nxt].k,
                                     wls[nxt].tol)
                femcg._check(rid)
                ids[rid] = nxt
                nxt += 1
            open_ = L.serve_step(srv)
            femcg._check(open_)
            for rid in list(ids):
                info = femcg.fem_request_info()
                i = ids[rid]
                X = np.zeros((nfree[i], wls[i].k)) if keep_x else None
                if L.serve_poll(srv, rid, femcg._np_ptr(X) if keep_x else None, C.byref(info)) == 1:
                    ids.pop(rid)
                    done[i] = dict(status=info.status, t_arr=t_arr[i], t_ready=info.t_ready - t_start,
                                   t_done=info.t_done - t_start, relres=info.relres_max)
                    if keep_x:
                        xs[i] = X
                    if len(done) % 25 == 0:
                        log("%s: %d of %d requests done at %.1f s" % (what, len(done), len(wls), now))
            if open_ == 0 and nxt < len(wls):
                time.sleep(max(0.0, min(0.01, t_arr[nxt] - (L.serve_clock(srv) - t_start))))
        L.serve_destroy(srv)
        if keep_x:
            done_cap.update(done)
        T = max(d["t_done"] for d in done.values())
        lat = [d["t_done"] - d["t_arr"] for d in done.values()]
        lat_s = [d["t_done"] - max(d["t_ready"], d["t_arr"]) for d in done.values()]
        bad = [i for i, d in done.items() if d["status"] != 0 or d["relres"] > wls[i].tol * 1.0001]
        return dict(solves_per_s=round(len(wls) / T, 3), wall_s=round(T, 3),
                    p50_ms=round(1e3 * percentile(lat, 50), 2), p99_ms=round(1e3 * percentile(lat, 99), 2),
                    p50_excl_assembly_ms=round(1e3 * percentile(lat_s, 50), 2),
                    p99_excl_assembly_ms=round(1e3 * percentile(lat_s, 99), 2), failed_or_above_tol=bad)

    base = np.array([r["t_arrival"] for r in reqs])
    cap = serve(np.zeros(len(wls)), keep_x=True, what="capacity run")
    capacity = cap["solves_per_s"]
    log("capacity (all submitted at t=0): %.3f solves/s in %.2f s" % (capacity, cap["wall_s"]))
    sweep = []
    for f in args.serve_fractions:
        rate = f * capacity
        r = serve(base / rate, what="trace at %.2fx capacity" % f)
        r.update(fraction=f, rate_per_s=round(rate, 3))
        sweep.append(r)
        log("rate %.2f/s (%.1fx capacity): %.3f solves/s, p50 %.0f ms, p99 %.0f ms"
            % (rate, f, r["solves_per_s"], r["p50_ms"], r["p99_ms"]))
    ref = min(args.serve_fractions, key=lambda f: abs(f - 0.7))
    t_ref = base / (ref * capacity)
    # one-at-a-time FP64 PCG on the same trace
    t_free, lat1, diff_fp64, solo = 0.0, [], [], []
    x1s = {}
    for i, w in enumerate(wls):
        ta = time.perf_counter()
        A = femcg.Matrix(w.mesh, w.order)
        B = torch.empty((A.n_free, w.k), dtype=torch.float64, device="cuda")
        X = torch.zeros_like(B)
        femcg.fem_rhs(A, gs[i], B)
        rc = femcg.pcg_solve(A, B, X, w.tol, femcg.default_opts(tol=w.tol, check_every=args.check_every))
        torch.cuda.synchronize()
        dur = time.perf_counter() - ta
        start = max(t_ref[i], t_free)
        t_free = start + dur
        lat1.append(t_free - t_ref[i])
        x1 = X.cpu().numpy()
        st1 = A.stats()
        solo.append(dict(rc=int(rc), iters=int(max(st1["iters"][:w.k])), relres=float(max(st1["relres"][:w.k]))))
        # per column, relative to that column's norm (columns differ in scale)
        diff_fp64.append(max(float(np.linalg.norm(xs[i][:, j] - x1[:, j]) / max(np.linalg.norm(x1[:, j]), 1e-300))
                             for j in range(w.k)))
        x1s[i] = x1
        if len(x1s) > 3:  # keep the largest differences' solutions only
            x1s.pop(min(x1s, key=lambda q: diff_fp64[q]))
        del A, B, X
        if (i + 1) % 25 == 0:
            log("one at a time: %d of %d requests" % (i + 1, len(wls)))
    # accuracy of the served solutions (capacity run):
    # (R) the oracle's Eq. (2) residual on a seeded random sample of the
    #     requests the oracle assembles in seconds (n_free <= 1.5M);
    # Eq. (1) error against the exact discrete solution where it is known
    #     (structured P1: the nodal values of the harmonic cubic data)
    import oracle
    rng = np.random.default_rng(7)
    eligible = [i for i in range(len(wls)) if nfree[i] <= 1500000]
    sample = sorted(rng.choice(eligible, size=min(args.serve_oracle_sample, len(eligible)), replace=False).tolist())
    t0 = time.time()
    rel_sample = []
    for i in sample:
        orc = oracle.System(wls[i].mesh, wls[i].order)
        rel_sample.append(float(orc.relres(orc.rhs(gs[i]), xs[i]).max()))
        del orc
        if len(rel_sample) % 10 == 0:
            log("oracle check: %d of %d sampled requests" % (len(rel_sample), len(sample)))
    log("oracle residual of %d sampled served solutions in %.1f s: max %.3e"
        % (len(sample), time.time() - t0, max(rel_sample) if rel_sample else float("nan")))
    # the largest served / one-at-a-time differences: both solutions against
    # the oracle's Eq. (2) residual (both pass tol => conditioning, not error)
    worst = []
    for i in sorted(x1s, key=lambda q: -diff_fp64[q]):
        rq = reqs[i]
        ent = dict(request=i, dim=rq["dim"], side=rq["m"], order=rq["order"], jitter=rq["jitter"], k=rq["k"],
                   n_free=nfree[i], diff=diff_fp64[i], served_relres_lib=done_cap[i]["relres"], one_at_a_time=solo[i])
        if nfree[i] <= 1500000:
            orc = oracle.System(wls[i].mesh, wls[i].order)
            bo = orc.rhs(gs[i])
            ent["oracle_relres_served"] = float(orc.relres(bo, xs[i]).max())
            ent["oracle_relres_one_at_a_time"] = float(orc.relres(bo, x1s[i]).max())
            del orc
        worst.append(ent)
        log("largest served vs one-at-a-time difference: %s" % json.dumps(ent))
    exact = [i for i in range(len(wls)) if wls[i].order == 1 and reqs[i]["jitter"] == 0.0]
    xerr = [max(float(np.linalg.norm(gs[i][f2ds[i], j] - xs[i][:, j]) / np.linalg.norm(gs[i][f2ds[i], j]))
                for j in range(wls[i].k)) for i in exact]
    main = [r for r in sweep if r["fraction"] == ref][0]
    line = {
        "metric": METRIC, "value": capacity, "unit": "solves/s", "n_gpus": 1,
        "steps": len(wls), "warmup": 0, "ms_per_step": round(1e3 / capacity, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-inner/f64-refined" if args.serve_mixed else "f64", "data": "synthetic",
        "config": {"workload": "c5_serving_stream", "recipe": " ".join((run_serve.__doc__ or "").split()),
                   "n_requests": len(wls), "slots": args.slots, "budget_gb": args.budget_gb,
                   "max2d": args.max2d, "max3d": args.max3d, "check_every": args.check_every},
        "capacity_run": cap,
        "latency_ms": {"rate_per_s": main["rate_per_s"], "fraction_of_capacity": ref, "p50": main["p50_ms"],
                       "p99": main["p99_ms"], "p50_excl_assembly": main["p50_excl_assembly_ms"],
                       "p99_excl_assembly": main["p99_excl_assembly_ms"]},
        "sweep": sweep,
        "one_at_a_time_fp64": {"rate_per_s": main["rate_per_s"], "solves_per_s": round(len(wls) / t_free, 3),
                               "p50_ms": round(1e3 * percentile(lat1, 50), 2),
                               "p99_ms": round(1e3 * percentile(lat1, 99), 2)},
        "accuracy": {
            "oracle_relres": {"sample": len(sample), "of_eligible": len(eligible),
                              "rule": "seeded random sample (numpy default_rng(7)) of the requests with "
                                      "n_free <= 1.5M; the oracle's own Eq. (2) residual of the served X",
                              "max": max(rel_sample) if rel_sample else None,
                              "all_within_tol": all(r <= 1.0001e-8 for r in rel_sample)},
            "x_err_vs_exact": {"requests": len(exact),
                               "rule": "structured P1 requests, whose exact discrete solution is the nodal "
                                       "harmonic data; Eq. (1), worst column per request",
                               "p50": percentile(xerr, 50) if xerr else None, "max": max(xerr) if xerr else None},
            "served_vs_one_at_a_time_fp64_rel_l2": {"p50": percentile(diff_fp64, 50), "max": max(diff_fp64),
                                                    "rule": "worst column per request, relative to its norm",
                                                    "largest": worst},
            "one_at_a_time_status": {"nonzero_rc": [i for i, q in enumerate(solo) if q["rc"] != 0]},
        },
    }
    print(json.dumps(line), flush=True)


def run_assembly(args):
    """Assembly of A = K_II and K_ID (Sect. 2.2 systems) on the host, on the
    device (FEM_ASSEMBLE_DEVICE) and by the oracle, for the C2-C4 meshes and
    3D P2 meshes of growing size; the device result is compared with the
    host result entry by entry (identical pattern, values to rounding)."""
    import numpy as np
    import torch

    import meshgen
    import oracle
    from paper_2201_05413_amd import femcg

    torch.cuda.set_device(0)
    cases = [("c2_2d_p1_jit_1024", meshgen.c2().mesh, 1), ("c3_3d_p1_128", meshgen.c3().mesh, 1),
             ("c4_2d_p2_jit_513", meshgen.c4().mesh, 2)]
    for m in args.asm_p2_sides:
        cases.append(("3d_p2_jit_%d" % m, meshgen.make_mesh(3, m, 0.3, 7), 2))
    rows = []
    for name, mesh, order in cases:
        # warm the device path once (first-use costs), then time both
        femcg.Matrix(meshgen.make_mesh(mesh["coords"].shape[1], 8, 0.0, 1), order,
                     femcg.FEM_FORMAT_SELL | femcg.FEM_ASSEMBLE_DEVICE).free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ad = femcg.Matrix(mesh, order, femcg.FEM_FORMAT_SELL | femcg.FEM_ASSEMBLE_DEVICE)
        t_dev = time.perf_counter() - t0
        t0 = time.perf_counter()
        Ah = femcg.Matrix(mesh, order, femcg.FEM_FORMAT_SELL)
        t_host = time.perf_counter() - t0
        rph, colh, valh = Ah.csr()
        rpd, cold, vald = Ad.csr()
        same = bool(np.array_equal(rph, rpd) and np.array_equal(colh, cold))
        rowmax = np.maximum.reduceat(np.abs(valh), rph[:-1])
        dmax = np.maximum.reduceat(np.abs(vald - valh), rph[:-1])
        rel = float((dmax / rowmax).max())
        row = dict(mesh=name, order=order, n_free=Ah.n_free, nnz=int(colh.size), host_s=round(t_host, 3),
                   device_s=round(t_dev, 3), speedup=round(t_host / t_dev, 2), pattern_identical=same,
                   max_row_rel_diff=rel)
        Ah.free()
        Ad.free()
        if Ah.n_free <= args.asm_oracle_max_n:
            t0 = time.perf_counter()
            oracle.System(mesh, order)
            row["oracle_s"] = round(time.perf_counter() - t0, 3)
        rows.append(row)
        log("assembly %s: n %d nnz %d host %.2f s device %.3f s (x%.1f), identical pattern %s, max row diff %.1e%s"
            % (name, row["n_free"], row["nnz"], t_host, t_dev, t_host / t_dev, same, rel,
               (", oracle %.2f s" % row["oracle_s"]) if "oracle_s" in row else ""))
    big = rows[-1]
    line = {
        "metric": "FEM assembly wall time, host vs device", "value": big["device_s"], "unit": "s",
        "n_gpus": 1, "steps": len(rows), "warmup": 1, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "assembly", "recipe": " ".join((run_assembly.__doc__ or "").split()),
                   "largest": big["mesh"]},
        "assembly": rows,
    }
    print(json.dumps(line), flush=True)


def run_degrees(args):
    """Polynomial degree study in the manner of Table 7 (Sect. 4.2): one 2D
    mesh of 294 x 294 vertices jittered by 0.3h (86,436 vertices; Table 7's
    mesh has 86,425), P1 to P4, Dirichlet data g = exp(x) cos(y) (harmonic,
    so u = g is the exact solution), tol 1e-12 (Table 7's epsilon).  Per
    degree: DOFs, structural nonzeros, assembly and tuner time, FP64 and
    mixed time-to-tol (median of the timed solves), iterations, the SpMM
    kernel's rate against the HBM roofline, the max nodal error against u,
    and the oracle's own residual of the FP64 solution."""
    import numpy as np
    import torch

    import meshgen
    import oracle
    from paper_2201_05413_amd import femcg

    torch.cuda.set_device(0)
    calibration_copy(args)
    mesh = meshgen.mesh2d(294, 0.3, 11)
    tol = 1e-12
    traffic = {}
    if args.traffic_json and os.path.exists(args.traffic_json):
        traffic = json.load(open(args.traffic_json))
    rows = []
    for order in args.degrees:
        t0 = time.perf_counter()
        A = femcg.Matrix(mesh, order, femcg.FEM_FORMAT_SELL | femcg.FEM_ASSEMBLE_DEVICE)
        t_asm = time.perf_counter() - t0
        t0 = time.perf_counter()
        fmt, cw, sg = femcg.fem_tune(A, 1, femcg.PCG_FP64)
        t_tune = time.perf_counter() - t0
        coords, _, f2d = A.dofs()
        g = (np.exp(coords[:, 0]) * np.cos(coords[:, 1]))[:, None]
        n = A.n_free
        B = torch.empty((n, 1), dtype=torch.float64, device="cuda")
        femcg.fem_rhs(A, g, B)
        res = {"mixed": dict(ms=None, iters=None)}
        precs = ((femcg.PCG_FP64, "fp64"),) if args.deg_fp64_only else ((femcg.PCG_FP64, "fp64"),
                                                                          (femcg.PCG_MIXED, "mixed"))
        for prec, key in precs:
            o = femcg.default_opts(tol=tol, precision=prec, check_every=args.check_every, inner_eta=args.eta)
            X = torch.zeros_like(B)
            femcg.pcg_solve(A, B, X, tol, o)  # warm-up (graph capture)
            ts = []
            for _ in range(max(1, args.steps)):
                X.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc = femcg.pcg_solve(A, B, X, tol, o)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                if rc != 0:
                    raise RuntimeError("P%d %s solve status %d" % (order, key, rc))
            st = A.stats()
            res[key] = dict(ms=round(1e3 * percentile(ts, 50), 3), iters=int(st["iters"][0]),
                            outer=int(st.get("outer", 0)), x=X.cpu().numpy())
        x = res["fp64"]["x"]
        err = float(np.abs(x[:, 0] - g[f2d, 0]).max())
        st = A.stats()
        nnz, nnz_nz = int(st["nnz"]), int(st["nnz_nonzero"])
        femcg.pcg_solve(A, B, torch.zeros_like(B), tol, femcg.default_opts(tol=tol))
        ms_k, by_k = femcg.pcg_time_kernel(A, 0, reps=args.kernel_reps)
        gbs = by_k / (ms_k * 1e-3) / 1e9
        row = dict(degree=order, dofs=int(len(coords)), n_free=n, nnz_structural=nnz, nnz_kept=nnz_nz,
                   assembly_s=round(t_asm, 3), device_assembled=bool(order <= 2), tune_s=round(t_tune, 3),
                   format=dict(sell=bool(fmt & femcg.FEM_FORMAT_SELL), C=cw, sigma=sg,
                               morton=bool(fmt & femcg.FEM_ORDER_SFC)),
                   fp64_ms=res["fp64"]["ms"], fp64_iters=res["fp64"]["iters"],
                   mixed_ms=res["mixed"]["ms"], mixed_inner_iters=res["mixed"]["iters"],
                   max_nodal_error=err, spmm_ms=round(ms_k, 5), spmm_gbs=round(gbs, 1),
                   spmm_frac=round(gbs / HBM_PEAK_GBS, 4), spmm_traffic=traffic.get("deg_p%d" % order))
        if not args.no_check:
            t0 = time.perf_counter()
            orc = oracle.System(mesh, order)
            bo = orc.rhs(g)
            row["oracle_relres_fp64"] = float(orc.relres(bo, x).max())
            if "x" in res["mixed"]:
                row["oracle_relres_mixed"] = float(orc.relres(bo, res["mixed"]["x"]).max())
            row["oracle_check_s"] = round(time.perf_counter() - t0, 2)
            del orc
        rows.append(row)
        log("P%d: dofs %d nnz %d | asm %.2f s tune %.2f s | fp64 %.2f ms (%d its) mixed %s ms | err %.2e | "
            "SpMM %.1f GB/s%s" % (order, row["dofs"], nnz, t_asm, t_tune, row["fp64_ms"], row["fp64_iters"],
                                  row["mixed_ms"] if row["mixed_ms"] is None else "%.2f" % row["mixed_ms"], err, gbs,
                                  (" | oracle relres %.2e / mixed %s" % (row["oracle_relres_fp64"],
                                   "%.2e" % row["oracle_relres_mixed"] if "oracle_relres_mixed" in row else "-"))
                                  if not args.no_check else ""))
        A.free()
    line = {
        "metric": "time-to-1e-12 residual per FEM degree (Table 7 analog)", "value": rows[-1]["fp64_ms"],
        "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (FP64 PCG) + f32-inner/f64-refined (mixed PCG)", "data": "synthetic",
        "config": {"workload": "degrees_2d_294_jit", "recipe": " ".join((run_degrees.__doc__ or "").split())},
        "degrees": rows,
    }
    print(json.dumps(line), flush=True)


def lumped_mass(mesh):
    """B of Sect. 2.2 for P1: the volume (area in 2D) of the cells incident
    at each vertex."""
    import numpy as np
    X = np.asarray(mesh["coords"], dtype=np.float64)
    T = np.asarray(mesh["cells"], dtype=np.int64)
    d = X.shape[1]
    J = np.stack([X[T[:, j + 1]] - X[T[:, 0]] for j in range(d)], axis=2)
    vol = np.abs(np.linalg.det(J)) / (2.0 if d == 2 else 6.0)
    B = np.zeros(len(X))
    for j in range(d + 1):
        np.add.at(B, T[:, j], vol)
    return B


def run_bicgstab(args):
    """The paper's solver (Sect. 3.2: BiCGStab + Block-Jacobi) against
    Jacobi-PCG on the C2 system (2D P1, 1024^2 jittered, column 0 of its
    data) and on C3's 128^3 Kuhn cube (column 0 of its data), tol 1e-8.
    BiCGStab runs with exact Block-Jacobi blocks of 1 (Jacobi), 4, 16 and 64
    consecutive free DOFs: iterations against block count, time to tol,
    algorithmic GB/s; the oracle recomputes each solution's residual.  Then
    the paper's nonsymmetric form A = B^-1 L (rows scaled by the inverse
    lumped volumes) with blocks of 1 and 4."""
    import numpy as np
    import torch

    import meshgen
    import oracle
    from paper_2201_05413_amd import femcg

    torch.cuda.set_device(0)
    rows = []
    for name, w in (("c2_2d_p1_jit_1024", meshgen.c2()), ("c3_3d_p1_128", meshgen.c3())):
        A = femcg.Matrix(w.mesh, w.order, femcg.FEM_FORMAT_SELL)
        fmt, cw, sg = femcg.fem_tune(A, 1, femcg.PCG_FP64)
        fname = "%s C%d sigma%d%s" % ("CSR" if (fmt & 0xf) == femcg.FEM_FORMAT_CSR else "SELL", cw, sg,
                                      " morton" if fmt & femcg.FEM_ORDER_SFC else "")
        log("%s: tuned format %s" % (name, fname))
        coords, _, _ = A.dofs()
        g = w.dirichlet(coords)[:, :1].copy()
        n = A.n_free
        B = torch.empty((n, 1), dtype=torch.float64, device="cuda")
        femcg.fem_rhs(A, g, B)
        orc = None if args.no_check else oracle.System(w.mesh, w.order)
        Bo = None if orc is None else orc.rhs(g)

        def check(X):
            return None if orc is None else float(orc.relres(Bo, X.cpu().numpy())[0])

        X = torch.zeros_like(B)
        o = femcg.default_opts(tol=w.tol, check_every=args.check_every)
        femcg.pcg_solve(A, B, X, w.tol, o)
        ts = []
        for _ in range(max(1, args.steps)):
            X.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            femcg.pcg_solve(A, B, X, w.tol, o)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        st = A.stats()
        rows.append(dict(system=name, n=n, solver="jacobi_pcg", format=fname, iters=int(st["iters"][0]),
                         ms=round(1e3 * percentile(ts, 50), 3), gbs=round(st["bytes"] / percentile(ts, 50) / 1e9, 1),
                         oracle_relres=check(X)))
        log("%s PCG: %d its, %.2f ms" % (name, rows[-1]["iters"], rows[-1]["ms"]))
        for bs in (1, 4, 16, 64):
            femcg.bicgstab_solve(A, B, X, w.tol, bs)  # warm-up: block inverses
            ts = []
            for _ in range(max(1, args.steps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, bst = femcg.bicgstab_solve(A, B, X, w.tol, bs)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                if rc != 0:
                    raise RuntimeError("%s BiCGStab bs %d status %d" % (name, bs, rc))
            t = percentile(ts, 50)
            rows.append(dict(system=name, n=n, solver="bicgstab_bj", form="K", format=fname, block_size=bs,
                             nblocks=int(bst["nblocks"]),
                             iters=int(bst["iters"]), restarts=int(bst["restarts"]), ms=round(1e3 * t, 3),
                             ms_per_iter=round(1e3 * t / max(1, bst["iters"]), 4),
                             gbs=round(bst["bytes"] / t / 1e9, 1), setup_s=round(bst["setup_s"], 3),
                             relres=bst["relres"], oracle_relres=check(X)))
            log("%s BiCGStab+BJ bs %d (%d blocks): %d its, %.2f ms (%.3f ms/it, %.0f GB/s)%s"
                % (name, bs, bst["nblocks"], bst["iters"], 1e3 * t, rows[-1]["ms_per_iter"], rows[-1]["gbs"],
                   "" if orc is None else ", oracle relres %.2e" % rows[-1]["oracle_relres"]))
        # the paper's nonsymmetric form A = B^-1 L (Sect. 2.2): rows scaled by
        # the inverse of B, the volume (area) of the cells around each vertex
        _, _, f2d = A.dofs()
        dsc = 1.0 / lumped_mass(w.mesh)[f2d]
        Ao = None
        if orc is not None:
            import scipy.sparse as sp
            rp, col, val = orc.A()
            Ao = sp.csr_matrix((val, col, rp), shape=(n, n))
        for bs in (1, 4):
            femcg.bicgstab_solve(A, B, X, w.tol, bs, row_scale=dsc)
            ts = []
            for _ in range(max(1, args.steps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, bst = femcg.bicgstab_solve(A, B, X, w.tol, bs, row_scale=dsc)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                if rc != 0:
                    raise RuntimeError("%s BiCGStab (B^-1 L) bs %d status %d" % (name, bs, rc))
            t = percentile(ts, 50)
            orel = None
            if Ao is not None:
                x, b0 = X.cpu().numpy()[:, 0], Bo[:, 0]
                orel = float(np.linalg.norm(dsc * (b0 - Ao @ x)) / np.linalg.norm(dsc * b0))
            rows.append(dict(system=name, n=n, solver="bicgstab_bj", form="B^-1 L", format=fname, block_size=bs,
                             nblocks=int(bst["nblocks"]), iters=int(bst["iters"]), restarts=int(bst["restarts"]),
                             ms=round(1e3 * t, 3), ms_per_iter=round(1e3 * t / max(1, bst["iters"]), 4),
                             gbs=round(bst["bytes"] / t / 1e9, 1), setup_s=round(bst["setup_s"], 3),
                             relres=bst["relres"], oracle_relres=orel))
            log("%s BiCGStab+BJ on B^-1 L, bs %d: %d its, %.2f ms (%.3f ms/it, %.0f GB/s)%s"
                % (name, bs, bst["iters"], 1e3 * t, rows[-1]["ms_per_iter"], rows[-1]["gbs"],
                   "" if orel is None else ", oracle relres (scaled) %.2e" % orel))
        del orc, Ao
        A.free()
    line = {
        "metric": "time-to-1e-8 residual, BiCGStab + Block-Jacobi vs Jacobi-PCG", "value": rows[1]["ms"],
        "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "bicgstab_bj", "recipe": " ".join((run_bicgstab.__doc__ or "").split())},
        "solves": rows,
    }
    print(json.dumps(line), flush=True)


def run_rhs(args):
    """The multiple right-hand-side model of Sect. 4.3 on one GPU: the
    iterative side T_IS(t) = T_IS_PC + t T_IS_SOLVE (Jacobi-PCG) against the
    direct side T_DS(t) = T_DS_FACT + t T_DS_SOLVE (sparse Cholesky,
    chol_factor / chol_solve), on C3's 128^3 Kuhn cube (the paper's Cube 1
    grid) and on the C2 system, t = 1, 2, 4, ..., 64 random harmonic
    right-hand sides (seed 3 / 8), PCG tolerances 1e-8 and 1e-12, each side
    solved one right-hand side at a time and as one block of t columns
    (Eq. (3)).  T_IS_PC is the Jacobi set-up (the solver copy with D^-1,
    rebuilt and uploaded); T_DS_FACT is the whole chol_factor (ordering,
    symbolic analysis, numeric factorisation); FEM assembly is common to both
    and left out.  T_IS_SOLVE and T_DS_SOLVE are least-squares slopes in t
    (blocks) or the one-column times (one at a time), and
    t_0 = (T_DS_FACT - T_IS_PC) / (T_IS_SOLVE - T_DS_SOLVE)."""
    import numpy as np
    import torch

    import meshgen
    import oracle
    from paper_2201_05413_amd import femcg

    torch.cuda.set_device(0)
    ts_all = sorted(set(args.rhs_ts) | {1})
    if ts_all[-1] > 64:
        raise SystemExit("--rhs-ts: at most 64 right-hand sides per block")
    tols = args.rhs_tols
    systems = [("c3_3d_p1_128", meshgen.mesh3d, 128, 3, 3), ("c2_2d_p1_jit_1024", lambda m: meshgen.c2().mesh, 0, 2, 8)]
    systems = [(nm, mk(m), d, sd) for nm, mk, m, d, sd in systems if nm[:2] in args.rhs_systems]
    reps = max(1, args.steps)
    out = []

    def timed(fn):
        tt = []
        for _ in range(reps):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - ta)
        return percentile(tt, 50)

    def slope(rows, key):
        tv = np.array([r["t"] for r in rows], dtype=float)
        yv = np.array([r[key] for r in rows])
        return float(np.polyfit(tv, yv, 1)[0])

    def t0_of(fact_s, pc_s, it_ms, ds_ms):
        den = it_ms - ds_ms
        return round((fact_s - pc_s) * 1e3 / den, 1) if den > 0 else None

    for name, mesh, dim, seed in systems:
        A = femcg.Matrix(mesh, 1, femcg.FEM_FORMAT_SELL)
        coords, _, _ = A.dofs()
        G = meshgen.harmonic_eval(meshgen.random_coeffs(dim, max(ts_all), seed), coords)
        n = A.n_free
        Ball = torch.empty((n, max(ts_all)), dtype=torch.float64, device="cuda")
        femcg.fem_rhs(A, np.ascontiguousarray(G), Ball)
        fmt, cw, sg = femcg.fem_tune(A, 1, femcg.PCG_FP64)
        # T_IS_PC: the Jacobi preconditioner lives in the solver copy (D^-1)
        t0 = time.perf_counter()
        femcg.fem_set_format(A, fmt, cw, sg)
        t_pc = time.perf_counter() - t0
        iterative = []
        orc = None
        for tol in tols:
            o = femcg.default_opts(tol=tol, check_every=args.check_every)

            def pcg(k):
                B = Ball[:, :k].contiguous()
                X = torch.zeros_like(B)
                femcg.pcg_solve(A, B, X, tol, o)  # warm-up (workspace, graph)

                def run():
                    X.zero_()
                    rc = femcg.pcg_solve(A, B, X, tol, o)
                    if rc != 0:
                        raise RuntimeError("%s k %d status %d" % (name, k, rc))
                tt = timed(run)
                return tt, int(max(A.stats()["iters"][:k])), X

            t1, it1, _ = pcg(1)
            rows = []
            for t in ts_all:
                tb, itb, Xb = pcg(t)
                rows.append(dict(t=t, block_ms=round(1e3 * tb, 3), block_ms_per_rhs=round(1e3 * tb / t, 3),
                                 block_iters_max=itb, one_at_a_time_ms=round(1e3 * t1 * t, 3)))
                log("%s tol %.0e t=%d: PCG block %.2f ms (%.2f per rhs, %d its), one at a time %.2f ms"
                    % (name, tol, t, 1e3 * tb, 1e3 * tb / t, itb, 1e3 * t1 * t))
            # parity: the oracle's Eq. (2) residual of the largest block
            if orc is None:
                orc = oracle.System(mesh, 1)
            rel_it = orc.relres(orc.rhs(G[:, :ts_all[-1]]), Xb.cpu().numpy())
            iterative.append(dict(tol=tol, iters_k1=it1, one_at_a_time_ms_per_rhs=round(1e3 * t1, 3),
                                  T_IS_SOLVE_block_ms=round(slope(rows, "block_ms"), 3),
                                  oracle_relres_max_largest_block=float(rel_it.max()), rows=rows))
        # the direct side
        L = femcg.Chol(A)
        cst = L.stats()
        log("%s: chol_factor %.3f s (ordering %.3f, symbolic and set-up %.3f, numeric %.3f), nnz(L) %.3g, %.3g flops"
            % (name, cst["total_s"], cst["order_s"], cst["symbolic_s"], cst["factor_s"], cst["nnz_l"], cst["flops"]))
        drows = []
        for t in ts_all:
            B = Ball[:, :t].contiguous()
            X = torch.empty_like(B)
            L.solve(B, X)
            td = timed(lambda: L.solve(B, X))
            drows.append(dict(t=t, block_ms=round(1e3 * td, 3), block_ms_per_rhs=round(1e3 * td / t, 3)))
            log("%s t=%d: direct block solve %.2f ms (%.3f per rhs)" % (name, t, 1e3 * td, 1e3 * td / t))
        d1 = drows[0]["block_ms"]
        for r in drows:
            r["one_at_a_time_ms"] = round(d1 * r["t"], 3)
        # parity: the oracle's Eq. (2) residual of the largest direct block
        if orc is None:
            orc = oracle.System(mesh, 1)
        rel = orc.relres(orc.rhs(G[:, :ts_all[-1]]), X.cpu().numpy())
        T_fact = cst["total_s"]
        T_ds_block = slope(drows, "block_ms")
        for it in iterative:
            it["t0_block"] = t0_of(T_fact, t_pc, it["T_IS_SOLVE_block_ms"], T_ds_block)
            it["t0_one_at_a_time"] = t0_of(T_fact, t_pc, it["one_at_a_time_ms_per_rhs"], d1)
        out.append(dict(system=name, n=n, T_IS_PC_s=round(t_pc, 3), iterative=iterative,
                        direct=dict(T_DS_FACT_s=round(T_fact, 3), order_s=round(cst["order_s"], 3),
                                    symbolic_s=round(cst["symbolic_s"], 3), numeric_s=round(cst["factor_s"], 3),
                                    nnz_l=cst["nnz_l"], flops=cst["flops"], max_front=cst["max_front"],
                                    factor_mb=round(cst["factor_mb"], 1),
                                    numeric_tflops=round(cst["flops"] / cst["factor_s"] / 1e12, 2),
                                    T_DS_SOLVE_block_ms=round(T_ds_block, 3), one_column_ms=d1,
                                    oracle_relres_max=float(rel.max()), rows=drows)))
        L.free()
        A.free()
    line = {
        "metric": "t_0 = (T_DS_FACT - T_IS_PC) / (T_IS_SOLVE - T_DS_SOLVE) (Sect. 4.3): Jacobi-PCG against sparse "
                  "Cholesky, blocks and one at a time",
        "value": out[0]["iterative"][0]["t0_block"], "unit": "right-hand sides", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "multi_rhs", "recipe": " ".join((run_rhs.__doc__ or "").split())},
        "systems": out,
    }
    print(json.dumps(line), flush=True)


def meshgen_doc(name):
    import meshgen
    f = {"c1": meshgen.c1, "c2": meshgen.c2, "c3": meshgen.c3, "c4": meshgen.c4}[name]
    return " ".join((f.__doc__ or "").split())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5", "asm", "deg", "bcg", "rhs"])
    ap.add_argument("--check-every", type=int, default=64)
    ap.add_argument("--format", default="auto", help="auto (tuner) | csr | sell:C:sigma")
    ap.add_argument("--order", default="natural", choices=["natural", "sfc"])
    ap.add_argument("--band", type=int, default=None, help="force tiling mode 0/1 (default: automatic)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--eta", type=float, default=1e-4)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--cold-mb", type=float, default=1200.0,
                    help="cold-cache SpMM: rotate copies of the matrix totalling at least this many MB "
                         "(0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle residual check (profiling runs)")
    ap.add_argument("--profile", type=int, default=0,
                    help="counter runs: FP64 solve capped at this many iterations, kernels timed, no JSON line")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--n-requests", type=int, default=200)
    ap.add_argument("--rhs-systems", nargs="+", default=["c3", "c2"], choices=["c3", "c2"],
                    help="rhs workload: the systems (the 128^3 cube, the C2 system)")
    ap.add_argument("--rhs-ts", type=int, nargs="+", default=[1, 2, 4, 8, 16, 32, 64],
                    help="rhs workload: block sizes t (1 is always run)")
    ap.add_argument("--rhs-tols", type=float, nargs="+", default=[1e-8, 1e-12],
                    help="rhs workload: PCG tolerances")
    ap.add_argument("--serve-oracle-sample", type=int, default=40,
                    help="c5: served solutions checked by the oracle's residual (seeded random sample)")
    ap.add_argument("--asm-p2-sides", type=int, nargs="*", default=[48, 96],
                    help="assembly timing: sides of the extra 3D P2 meshes")
    ap.add_argument("--asm-oracle-max-n", type=int, default=3000000,
                    help="assembly timing: time the oracle's assembly up to this many free DOFs")
    ap.add_argument("--degrees", type=int, nargs="+", default=[1, 2, 3, 4], help="deg workload: FEM degrees")
    ap.add_argument("--deg-fp64-only", action="store_true", help="deg workload: skip the mixed solves (counter runs)")
    ap.add_argument("--serve-fractions", type=float, nargs="+", default=[0.5, 1.0],
                    help="serving: arrival rates as fractions of the measured capacity")
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--max2d", type=int, default=1024)
    ap.add_argument("--max3d", type=int, default=96)
    ap.add_argument("--serve-mixed", action="store_true")
    ap.add_argument("--calibrate-copy-mb", type=float, default=0.0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the row-block sharding over several GPUs is designed, "
              "not built; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c5":
        run_serve(args)
    elif args.workload == "asm":
        run_assembly(args)
    elif args.workload == "deg":
        run_degrees(args)
    elif args.workload == "bcg":
        run_bicgstab(args)
    elif args.workload == "rhs":
        run_rhs(args)
    else:
        run_single(args)


if __name__ == "__main__":
    main()
