"""Benchmark: time-to-solution of MINRES-CG on one MI355X.

A step is one complete solve A x = b to an FP64 true relative residual of
1e-8 (outer MINRES always FP64).  Default workload: the FE-elasticity-like
27-point system, 80^3 nodes x 3 dof (n = 1,536,000, nnz = 121,331,448),
shifted to 30 negative eigenvalues.  Legs, all on the same handle type and
right-hand side:
  * learned + mixed: inner CG in FP32 with the learned C C^T (network trained
    at setup on smaller matrices of the same family) -- `value`;
  * mixed with the IC-style incomplete LDL^T(0), mixed with Jacobi;
  * FP64 with LDL^T(0), and plain FP64 with Jacobi (the method without the
    additions: the denominator of the speedup).
Printed JSON line: metric/value/unit (seconds per solve, lower is better),
every leg, a roofline object for the headline leg's dominant kernel (the
product with A inside the learned iteration, timed with HIP events on the
solve stream around each of its launches), SpMV rates on this matrix and on
the 128^3 7-point Laplacian, and a CPU baseline: the FP64 oracle timed on a
bounded sample of the same workload.  --oracle-x adds a full oracle solve and
every leg's distance to its solution.  --workload laplace3d / batched run the
3D Laplacian and the batched shifted-systems workloads.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# HBM bytes per launch of a roofline kernel (FP32 inner) from FETCH_SIZE /
# WRITE_SIZE counter runs, scaled by the factors a plain copy of known size
# gives, keyed by (workload, kernel); the counter tables are in profiles/
# (cg_update_laplace3d_128_k20.md for the update kernel).  Valid only while
# those kernels are unchanged: drop an entry after changing its kernel.
MMR_TRAFFIC_BYTES = {("laplace3d_rand_128x128x128_k20", "update_v"): 226.9e6}
TRAFFIC_BYTES = {("fe27_80^3x3_k30", "bsell_spmv_f32"): 600.6e6}   # profiles/fe27_80_k30.md


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name, m, device):
    from paper_1805_12417_amd import workloads as W
    if name == "laplace3d":
        return W.shifted_laplace3d(m=m or 128, k=20, device=device, verbose=True)
    if name == "laplace2d":
        return W.shifted_laplace2d()
    if name == "fe27":
        return W.shifted_fe27(m=m or 80, k=30, device=device, verbose=True)
    raise SystemExit("unknown workload " + name)


def sell_shape(w):
    """(padded entries, slices) of A's sliced ELL copy: slices of 64 rows,
    each padded to its longest row."""
    ln = np.diff(w.row_ptr)
    ns = (w.n + 63) // 64
    pad = np.zeros(ns * 64, ln.dtype)
    pad[:w.n] = ln
    return int(64 * pad.reshape(ns, 64).max(axis=1).sum()), ns


def spmv_bytes(w, elem, block=0, sell=0):
    """Bytes y = A x must move in the storage used: values, indices, row (or
    slice) pointers, x read once, y written.  block = bs: block CSR (one index
    per bs^2 values, block-row pointers); sell = column bits of the sliced
    ELL copy (padded entries, 8-byte slice offsets)."""
    if block:
        nnzb = w.nnz // (block * block)
        return w.nnz * elem + 4 * nnzb + 4 * (w.n // block + 1) + 2 * w.n * elem
    if sell:
        P, ns = sell_shape(w)
        return P * (elem + sell // 8) + 8 * (ns + 1) + 2 * w.n * elem
    return w.nnz * (elem + 4) + 4 * (w.n + 1) + 2 * w.n * elem


def mmr_bytes(w, elem, block=0, sell=0):
    """Bytes one M_mr apply must move: A in the storage used (as spmv_bytes),
    plus Vhat read once."""
    return spmv_bytes(w, elem, block, sell) + w.n * w.k * elem


def time_solves(s, pc, b, steps, warmup, rtol, rtol_in):
    import torch
    for _ in range(warmup):
        s.solve(b, pc, rtol_out=rtol, rtol_in=rtol_in)
    torch.cuda.synchronize()
    if s.precision is not None:
        try:
            s.kernel_time(reset=True)
        except Exception:
            pass
    t0 = time.perf_counter()
    stats = []
    for _ in range(steps):
        x, st = s.solve(b, pc, rtol_out=rtol, rtol_in=rtol_in)
        stats.append(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, x, stats


def median_flushed(s, pc, b, rtol, rtol_in, reps=5, flush_mb=512):
    """Median of `reps` solves, each timed with HIP events on its own after a
    read of a flush_mb buffer (the caches hold none of the solve's data at
    its start)."""
    import torch
    buf = torch.ones(flush_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        float(buf.sum())
        torch.cuda.synchronize()
        e0.record()
        s.solve(b, pc, rtol_out=rtol, rtol_in=rtol_in)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del buf
    return float(np.median(ts))


def time_spmv(s, precision, w, reps=50):
    import torch
    dt = torch.float64 if precision == 0 else torch.float32
    x = torch.randn(w.n, dtype=dt, device="cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(5):
        s.spmv(x, precision, out=y)
    e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        s.spmv(x, precision, out=y)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(w, gpu_inner_its, gpu_outer_its, rtol, rtol_in, budget_s=30.0):
    """The FP64 oracle's MINRES-CG (Jacobi second level) on the full system,
    timed end to end on the host cores.  A cap on the total inner iterations
    bounds the work to about budget_s seconds (calibrated on 3 iterations);
    when the cap stops the solve first, the time is scaled by the inner
    iteration count of the FP64 GPU solve.  Returns (baseline dict, oracle
    result dict: x and its statistics)."""
    import oracle as O
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    pc = O.InnerPC(O.PC_JACOBI, P)
    y = np.random.default_rng(0).standard_normal(w.n)
    t0 = time.perf_counter()
    O.pcg(P, pc, y, rtol=0.0, maxit=3)
    per_it = max(time.perf_counter() - t0, 1e-4) / 3
    cap = int(max(8, budget_s / per_it))
    t0 = time.perf_counter()
    r = O.minres_cg(P, pc, w.b, rtol_out=rtol, rtol_in=rtol_in, maxit_in_total=cap)
    dt = time.perf_counter() - t0
    done = max(1, r["inner_its_total"])
    full = r["status"] == O.OK
    est = dt if full else dt * gpu_inner_its / done
    model, ncpu = cpu_info()
    if full:
        sample = ("complete FP64 oracle MINRES-CG solve (Jacobi second level) of the full "
                  "system to the same tolerance: %d outer / %d inner iterations, %.2f s" % (
                      r["outer_its"], done, dt))
    else:
        sample = ("FP64 oracle MINRES-CG (Jacobi) on the full system, stopped by a cap of %d "
                  "inner CG iterations (%d outer, %.2f s timed), scaled to the %d inner "
                  "iterations of the FP64 GPU solve (%d outer)" % (
                      cap, r["outer_its"], dt, gpu_inner_its, gpu_outer_its))
    return dict(value=round(est, 3), unit="s", cores=O.num_threads(), kind="oracle",
                cpu_model=model, nproc=ncpu, timed_seconds=round(dt, 3), complete_solve=full,
                oracle_status=r["status"], oracle_final_relres=r["final_relres"],
                sample=sample), r


def oracle_solution(w, rtol, rtol_in):
    """Full FP64 oracle solve (Jacobi second level) of w; (x, result dict, s)."""
    import oracle as O
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    t0 = time.perf_counter()
    r = O.minres_cg(P, O.InnerPC(O.PC_JACOBI, P), w.b, rtol_out=rtol, rtol_in=rtol_in)
    return r["x"], r, time.perf_counter() - t0


def laplace_spmv_rates(device, m=128):
    """SpMV rates on the 128^3 7-point random-coefficient Laplacian (the
    unshifted operator: the shift changes diagonal values only, not a byte
    moved), FP32 and FP64, in the sliced ELL storage the solver picks."""
    import torch
    from paper_1805_12417_amd import solver as S
    from paper_1805_12417_amd import workloads as W
    A = W.laplace3d_random(m, m, m, np.random.default_rng(2))
    A.sort_indices()
    wk = W.Workload("laplace3d_%d" % m, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                    A.data.astype(np.float64), np.zeros(A.shape[0]),
                    np.zeros((A.shape[0], 0), order="F"), np.zeros(0), 0.0, {})
    out = {}
    for prec, key, elem in ((S.PREC_MIXED, "fp32", 4), (S.PREC_FP64, "fp64", 8)):
        s, _ = S.from_workload(wk, precision=prec, device=device)
        ms = time_spmv(s, 1 if prec == S.PREC_MIXED else 0, wk)
        nbytes = spmv_bytes(wk, elem, s.block_csr, s.sliced_ell)
        out[key + "_us"] = round(ms * 1e3, 2)
        out[key + "_GBps"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
        out[key + "_frac"] = round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
        s.close()
    out.update(n=wk.n, nnz=wk.nnz, storage="sliced ELL, 16-bit column offsets")
    del A
    return out


def train_learned(args, k, log):
    """The learned factor's weights: one network trained on 16 seeded
    instances of the FE-like family (16^3 nodes x 3 dof, k = 6, seeds
    5000-5015, never the benchmark matrix's seed), 1,280 pairs y = M_mr z
    each (20,480 in all), Adam."""
    from paper_1805_12417_amd import learned as LL
    from paper_1805_12417_amd import workloads as W
    t1 = time.perf_counter()
    fam = [W.shifted_fe27(m=16, k=6, seed=5000 + i, device="cuda") for i in range(16)]
    t_gen = time.perf_counter() - t1
    log("learned: 16 training matrices (16^3 nodes x 3) in %.1fs" % t_gen)
    theta, hist, t_train = LL.fit(fam, block_size=3, pairs_per_matrix=1280,
                                  steps=args.train_steps, log=log)
    info = dict(train_s=round(t_train, 2), train_matrices_s=round(t_gen, 2),
                train_loss_final=float(np.mean(hist[-50:])), train_steps=args.train_steps,
                train_matrices="16 x fe27 16^3 nodes x 3 dof, k = 6, seeds 5000-5015, "
                               "20,480 pairs y = M_mr z")
    return theta, info


def bench_fe27(args):
    """FE-like 27-point system (80^3 nodes x 3 dof, k = 30): learned C C^T,
    the IC-style incomplete LDL^T(0) (8-colour node sweeps) and Jacobi in
    mixed precision (FP32 inner / FP64 outer), FP64 with LDL^T(0), and plain
    FP64 with Jacobi."""
    import torch
    from paper_1805_12417_amd import learned as LL
    from paper_1805_12417_amd import solver as S
    t0 = time.perf_counter()
    w = make_workload("fe27", args.m, "cuda")
    log("workload %s n=%d nnz=%d k=%d setup %.1fs" % (w.name, w.n, w.nnz, w.k,
                                                     time.perf_counter() - t0))
    legs = [(S.PREC_MIXED, "learned"), (S.PREC_MIXED, "ildl0"), (S.PREC_MIXED, "jacobi"),
            (S.PREC_FP64, "ildl0"), (S.PREC_FP64, "jacobi")]
    if args.no_learned:
        legs = legs[1:]
    if args.legs:   # a subset (profiling runs); the JSON line then lacks the missing legs
        keep = args.legs.split(",")
        legs = [lg for lg in legs if "%s_%s" % ("mixed" if lg[0] == S.PREC_MIXED else "fp64",
                                                  lg[1]) in keep]
    fac = None
    learned_info = {}
    if not args.no_learned:
        theta, learned_info = train_learned(args, w.k, log)
        dev = torch.device("cuda")
        fac = LL.LearnedFactor(torch.from_numpy(w.row_ptr).to(dev),
                               torch.from_numpy(w.col).to(dev),
                               torch.from_numpy(w.val).to(dev), block_size=3, theta=theta)
    res, xs = {}, {}
    for prec, pcname in legs:
        s, b = S.from_workload(w, precision=prec, autotune=True)
        t1 = time.perf_counter()
        pc = fac.preconditioner(s) if pcname == "learned" else s.preconditioner(pcname)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t1
        dt, x, st = time_solves(s, pc, b, args.steps, args.warmup, args.rtol, args.rtol_in)
        rr = b - s.spmv(x)
        relres = float(torch.linalg.vector_norm(rr) / torch.linalg.vector_norm(b))
        key = "%s_%s" % ("mixed" if prec == S.PREC_MIXED else "fp64", pcname)
        res[key] = dict(seconds=round(dt, 4), outer_its=st[-1].outer_its,
                        inner_its_total=st[-1].inner_its_total, final_relres_fp64=relres,
                        status=st[-1].status_name, precond_setup_s=round(setup, 3))
        if key in ("mixed_learned", "fp64_jacobi") and not args.legs:
            res[key]["median5_flushed_s"] = round(
                median_flushed(s, pc, b, args.rtol, args.rtol_in), 4)
        xs[key] = x.cpu().numpy()
        if pcname == "jacobi":
            ip = 1 if prec == S.PREC_MIXED else 0
            ms = time_spmv(s, ip, w)
            nbytes = spmv_bytes(w, 4 if ip else 8, s.block_csr, s.sliced_ell)
            res[key]["spmv"] = dict(us=round(ms * 1e3, 2),
                                    GBps=round(nbytes / (ms * 1e-3) / 1e9, 1),
                                    frac=round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                                    block=s.block_csr, bytes=nbytes)
            log("  spmv %s: %.1f us, %.0f GB/s (block %d)" % (key, ms * 1e3,
                                                             nbytes / (ms * 1e-3) / 1e9,
                                                             s.block_csr))
        log("%s: %.3f s/solve %s outer=%d inner=%d relres=%.2e (precond setup %.2fs)" % (
            key, dt, st[-1].status_name, st[-1].outer_its, st[-1].inner_its_total, relres, setup))
        pc.close()
        s.close()
    head_key = "mixed_learned" if fac is not None else "mixed_ildl0"
    if fac is not None:
        res["mixed_learned"].update(learned_info)
        res["mixed_learned"]["network_forward_ms"] = round(fac.forward_ms(), 3)

    # roofline of the headline leg's dominant kernel: the product with A (Ap
    # with p^T A p, sliced 3 x 3 block copy, FP32), HIP events around each
    # launch on the solve stream, launches after an inner stop excluded
    sprof, b = S.from_workload(w, precision=S.PREC_MIXED, autotune=True, profile=2)
    pcp = fac.preconditioner(sprof) if fac is not None else sprof.preconditioner("ildl0")
    dt_prof, _, _ = time_solves(sprof, pcp, b, args.steps, args.warmup, args.rtol, args.rtol_in)
    kms, klaunch = sprof.kernel_time()
    bs = sprof.block_csr
    xcd = sprof.xcd_sections
    pcp.close()
    sprof.close()
    avg_ms = kms / max(klaunch, 1)
    bytes_k = spmv_bytes(w, 4, bs, 0)
    achieved = bytes_k / (avg_ms * 1e-3) / 1e9
    kname = ("k_bsell_spmv<3, float, true, float>: A p with per-block p^T A p over the sliced "
             "3 x 3 block copy of A (FP32 values, one int32 block column per block)")
    roofline = dict(bound="hbm", kernel=kname, achieved=round(achieved, 1), peak=HBM_PEAK_GBPS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBPS, 4),
                    traffic=TRAFFIC_BYTES.get((w.name, "bsell_spmv_f32")),
                    avg_launch_us=round(avg_ms * 1e3, 2), launches=klaunch,
                    algorithmic_bytes=bytes_k, xcd_sections=xcd,
                    bytes_model="4 nnz (values) + 4 nnz/9 (block columns) + 4 (n/3 + 1) + "
                                "2 x 4n (x read, y written)",
                    solve_s_with_events=round(dt_prof, 4))
    log("roofline: %.1f us per launch (%d launches), %.0f GB/s = %.3f of peak, XCD slice "
        "sections %d" % (avg_ms * 1e3, klaunch, achieved, achieved / HBM_PEAK_GBPS, xcd))
    if fac is not None:
        fac.close()

    lap = None
    if not args.no_laplace_spmv and not args.legs:
        lap = laplace_spmv_rates("cuda")
        log("laplace3d 128^3 spmv: fp32 %.1f us %.0f GB/s, fp64 %.1f us %.0f GB/s" % (
            lap["fp32_us"], lap["fp32_GBps"], lap["fp64_us"], lap["fp64_GBps"]))

    cpu, ro = None, None
    if not args.no_cpu and not args.legs:
        ref = res["fp64_jacobi"]
        cpu, ro = cpu_baseline(w, ref["inner_its_total"], ref["outer_its"], args.rtol,
                               args.rtol_in, args.cpu_budget)
        log("cpu baseline: %.2f s (timed %.1f s, complete %s), %d threads" % (
            cpu["value"], cpu["timed_seconds"], cpu["complete_solve"], cpu["cores"]))
        if not cpu["complete_solve"]:
            ro = None
    oracle_x = None
    if ro is None and args.oracle_x:
        xo_, ro, t_o = oracle_solution(w, args.rtol, args.rtol_in)
    if ro is not None:
        import oracle as O
        xo = ro["x"]
        no = float(np.linalg.norm(xo))
        oracle_x = dict(status=ro["status"], outer_its=ro["outer_its"],
                        inner_its_total=ro["inner_its_total"], final_relres=ro["final_relres"],
                        note="x_err_vs_oracle of each leg is |x - x_oracle| / |x_oracle|; "
                             "x_err_bound = (r_leg + r_oracle) ||b|| / min|lambda(A)| / "
                             "|x_oracle|, the bound any two solutions with these residuals obey")
        bn = float(np.linalg.norm(w.b))
        for key, x in xs.items():
            res[key]["x_err_vs_oracle"] = float(np.linalg.norm(x - xo) / no)
            res[key]["x_err_bound"] = float((res[key]["final_relres_fp64"] + ro["final_relres"]) *
                                            bn / w.meta["min_abs_eig"] / no)
        log("errors vs the oracle: %s" % ({k: "%.2e" % v["x_err_vs_oracle"]
                                             for k, v in res.items()}))
    if args.legs:
        print(json.dumps({"legs": res, "roofline": roofline}), flush=True)
        return
    head = res[head_key]
    base = res["fp64_jacobi"]
    out = {"metric": "time-to-1e-8 FP64 relative residual, learned+mixed MINRES-CG vs plain FP64",
           "value": head["seconds"], "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(head["seconds"] * 1e3, 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 inner (C, C^T stored f16) / f64 outer", "data": "synthetic",
           "config": {"workload": w.name, "n": w.n, "nnz": w.nnz, "k": w.k,
                      "rtol_out": args.rtol, "rtol_in": args.rtol_in,
                      "precond": "learned C C^T" if fac is not None else "ildl0",
                      "parallelism": "none"},
           "outer_its": head["outer_its"], "inner_its_total": head["inner_its_total"],
           "final_relres_fp64": head["final_relres_fp64"], "status": head["status"],
           "speedup_vs_plain_fp64": round(base["seconds"] / head["seconds"], 3),
           "speedup_median5_flushed": (round(base["median5_flushed_s"] /
                                             head["median5_flushed_s"], 3)
                                       if "median5_flushed_s" in head and
                                       "median5_flushed_s" in base else None),
           "speedup_vs_fp64_ildl0": round(res["fp64_ildl0"]["seconds"] / head["seconds"], 3),
           "speedup_vs_mixed_ildl0": round(res["mixed_ildl0"]["seconds"] / head["seconds"], 3),
           "runs": res,
           "spmv_fe27": dict(fp32=res.get("mixed_jacobi", {}).get("spmv"),
                             fp64=base.get("spmv")),
           "spmv_laplace3d_128": lap,
           "roofline": roofline,
           "cpu_baseline": cpu,
           "oracle_solution": oracle_x}
    print(json.dumps(out), flush=True)


def bench_brake(args):
    """Disk-brake inner-level systems (Section 3.1): K_E - |gamma|^2 M on the
    FE-like stiffness (m^3 nodes x 3 dof, default 48^3: n = 331,776) with a
    lumped mass matrix, k = 18 negative eigenvalues (the paper's small brake
    model has 18), and a sweep of 8 shifts gamma of the same modulus.  The
    setup -- the k negative eigenpairs on the GPU (the library's
    Chebyshev-filtered subspace iteration) and the second-level
    preconditioner -- is done once and reused by every solve of the sweep;
    a step is the whole sweep (8 solves to 1e-8)."""
    import torch
    from paper_1805_12417_amd import solver as S
    from paper_1805_12417_amd import workloads as W
    t0 = time.perf_counter()
    m = args.m or 48
    w = W.brake_inner_level(m=m, k=18, device="cuda", verbose=False)
    sweep = W.brake_sweep_rhs(w, 8, 11)
    log("brake inner level n=%d nnz=%d k=%d |gamma|^2=%.4g, generated in %.1fs" % (
        w.n, w.nnz, w.k, w.meta["gamma_abs2"], time.perf_counter() - t0))
    dev = torch.device("cuda")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (w.row_ptr, w.col, w.val))
    Bs = [torch.from_numpy(b).to(dev) for _, b in sweep]
    legs = {}
    for prec, pcname in ((S.PREC_MIXED, "ildl0"), (S.PREC_MIXED, "jacobi"),
                         (S.PREC_FP64, "jacobi")):
        key = "%s_%s" % ("mixed" if prec == S.PREC_MIXED else "fp64", pcname)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lam, V, est = S.lowest_eigs(rp, ci, va, w.k, tol=1e-10)     # setup stage 2 on the GPU
        s = S.MinresCG(rp, ci, va, V.contiguous(), torch.from_numpy(lam).to(dev),
                       precision=prec, block_size=3, autotune=True)
        pc = s.preconditioner(pcname)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t1
        for _ in range(args.warmup):
            s.solve(Bs[0], pc, rtol_out=args.rtol, rtol_in=args.rtol_in)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        worst, its = 0.0, []
        for _ in range(args.steps):
            for b in Bs:
                x, st = s.solve(b, pc, rtol_out=args.rtol, rtol_in=args.rtol_in)
                its.append(st.inner_its_total)
                if st.status != 0:
                    raise RuntimeError("brake %s: status %s" % (key, st.status_name))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        for b in Bs:   # FP64 true residuals of the last step's solutions
            x, _ = s.solve(b, pc, rtol_out=args.rtol, rtol_in=args.rtol_in)
            r = b - s.spmv(x)
            worst = max(worst, float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)))
        legs[key] = dict(sweep_s=round(dt, 4), per_solve_s=round(dt / len(Bs), 4),
                         setup_s=round(setup, 3), eig_outer_its=est["outer_its"],
                         eig_max_lam_diff=float(np.abs(lam - w.lam).max()),
                         inner_its_mean=float(np.mean(its)), worst_relres_fp64=worst)
        log("brake %s: sweep of %d solves %.3f s (%.4f s each), setup %.2f s (eigs %d outer), "
            "inner its %.0f, worst relres %.2e" % (key, len(Bs), dt, dt / len(Bs), setup,
                                                  est["outer_its"], np.mean(its), worst))
        pc.close()
        s.close()
    best = min(legs, key=lambda k: legs[k]["sweep_s"])
    head = legs[best]
    out = {"metric": "time to solve a sweep of 8 brake inner-level systems (one |gamma|) to 1e-8",
           "value": head["sweep_s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * head["sweep_s"], 2),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 inner / f64 outer", "data": "synthetic",
           "config": {"workload": w.name, "n": w.n, "nnz": w.nnz, "k": w.k, "shifts": len(Bs),
                      "gamma_abs2": w.meta["gamma_abs2"], "rtol_out": args.rtol,
                      "rtol_in": args.rtol_in, "leg": best},
           "legs": legs,
           "speedup_vs_plain_fp64": round(legs["fp64_jacobi"]["sweep_s"] / head["sweep_s"], 3)}
    print(json.dumps(out), flush=True)


def ildlp_levels(f):
    """Depth of the level schedule of a unit lower triangular factor."""
    n = f["perm"].size
    lev = np.zeros(n, np.int64)
    lp, lc = f["l_ptr"], f["l_col"]
    for i in range(n):
        if lp[i + 1] > lp[i]:
            lev[i] = lev[lc[lp[i]:lp[i + 1]]].max() + 1
    return int(lev.max()) + 1 if n else 0


def bench_kkt(args):
    """Saddle-point systems [[K, B^T], [B, 0]] (K the 2D Laplacian on m x m,
    default m = 128, 64 constraint rows of 6 unknowns each, interleaved):
    the zero diagonal rules out Jacobi and gives the unpivoted ILDL^T(0) zero
    pivots, so the second level is the pivoted ILDL^T(fill, drop) of
    Section 4 (fill 3, drop 1e-3, the defaults Section 4.3 names), applied
    exactly or with 3 Jacobi sweeps per triangle, or none.  A step is one
    solve to 1e-8; the factorization is setup, timed apart.  value: the
    fastest leg."""
    import torch
    import oracle as O
    from paper_1805_12417_amd import solver as S
    from paper_1805_12417_amd import workloads as W
    t0 = time.perf_counter()
    m = args.m or 128
    w = W.kkt_saddle(m=m, n_con=64, seed=21, coupling=10.0, device="cuda")
    log("kkt n=%d nnz=%d k=%d min|eig|=%.3g, generated in %.1fs" % (
        w.n, w.nnz, w.k, w.meta["min_abs_eig"], time.perf_counter() - t0))
    fill, drop = 3.0, 1e-3
    legs = {}
    fact = None
    for prec, pcname, sw in ((S.PREC_MIXED, "ildlp", 3), (S.PREC_FP64, "ildlp", 3),
                             (S.PREC_MIXED, "ildlp", 0), (S.PREC_FP64, "ildlp", 0),
                             (S.PREC_MIXED, "none", 0), (S.PREC_FP64, "none", 0)):
        key = "%s_%s%s" % ("mixed" if prec == S.PREC_MIXED else "fp64", pcname,
                           "_sweeps%d" % sw if sw else "")
        if args.legs and key not in args.legs.split(","):
            continue
        s, b = S.from_workload(w, precision=prec, autotune=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pc = s.preconditioner(pcname, fill=fill, drop=drop, sweeps=sw)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t1
        if pcname == "ildlp" and fact is None:
            fact = pc.ildlp_factor()
        for _ in range(args.warmup):
            s.solve(b, pc, rtol_out=args.rtol, rtol_in=args.rtol_in)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            x, st = s.solve(b, pc, rtol_out=args.rtol, rtol_in=args.rtol_in)
            if st.status != 0:
                raise RuntimeError("kkt %s: status %s" % (key, st.status_name))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        r = b - s.spmv(x)
        rel = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))
        legs[key] = dict(s_per_solve=round(dt, 4), setup_s=round(setup, 3),
                         outer_its=st.outer_its, inner_its=st.inner_its_total,
                         us_per_inner_it=round(1e6 * dt / max(1, st.inner_its_total), 2),
                         relres_fp64=rel, x=x.cpu().numpy())
        log("kkt %s: %.4f s/solve, setup %.3f s, %d outer / %d inner its (%.1f us each), "
            "relres %.2e" % (key, dt, setup, st.outer_its, st.inner_its_total,
                             1e6 * dt / max(1, st.inner_its_total), rel))
        pc.close()
        s.close()
    # the Jacobi and unpivoted routes
    s, _ = S.from_workload(w)
    try:
        s.preconditioner("jacobi")
        jac = "accepted"
    except S.MCGError as e:
        jac = "rejected: %s" % N_name(e)
    s.close()
    if fact is None:
        s, _ = S.from_workload(w)
        pc = s.preconditioner("ildlp", fill=fill, drop=drop)
        fact = pc.ildlp_factor()
        pc.close()
        s.close()
    levels = ildlp_levels(fact)
    # host oracle: the same factor and a complete solve
    cpu = None
    if not args.no_cpu:
        t1 = time.perf_counter()
        F = O.ILDLP(w.row_ptr, w.col, w.val, fill=fill, drop=drop)
        tf = time.perf_counter() - t1
        P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
        t1 = time.perf_counter()
        ro = O.minres_cg(P, O.InnerPC(O.PC_ILDLP, factor=F, sweeps=3), w.b,
                         rtol_out=args.rtol, rtol_in=args.rtol_in)
        ts = time.perf_counter() - t1
        model, ncpu = cpu_info()
        cpu = {"value": round(ts, 3), "unit": "s", "cores": O.num_threads(), "kind": "oracle",
               "cpu_model": model, "nproc": ncpu,
               "sample": "complete FP64 oracle MINRES-CG solve with the oracle's own ILDLP factor, "
                         "3 Jacobi sweeps per triangle (factorization %.2f s apart, one thread), "
                         "%d outer / %d inner its" % (
                             tf, ro["outer_its"], ro["inner_its_total"])}
        for key, leg in legs.items():
            leg["x_err_vs_oracle"] = float(np.linalg.norm(leg["x"] - ro["x"]) /
                                           np.linalg.norm(ro["x"]))
    for leg in legs.values():
        leg.pop("x")
    best = min(legs, key=lambda k: legs[k]["s_per_solve"])
    head = legs[best]
    out = {"metric": "time to solve one saddle-point system to 1e-8 (FP64 true residual)",
           "value": head["s_per_solve"], "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * head["s_per_solve"], 2),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 inner / f64 outer", "data": "synthetic",
           "config": {"workload": w.name, "n": w.n, "nnz": w.nnz, "k": w.k, "fill": fill,
                      "drop": drop, "nnz_L": int(fact["l_val"].size),
                      "two_by_two_pivots": int((fact["bsize"] == 2).sum()),
                      "levels": levels, "rtol_out": args.rtol, "rtol_in": args.rtol_in,
                      "leg": best},
           "legs": legs, "jacobi": jac, "cpu_baseline": cpu,
           "speedup_vs_no_second_level": (round(legs["mixed_none"]["s_per_solve"] /
                                                head["s_per_solve"], 3)
                                          if "mixed_none" in legs else None)}
    print(json.dumps(out), flush=True)


def bench_laplace2d(args):
    """The 64 x 64 2D Laplacian shifted to 6 negative eigenvalues with the
    closed-form eigenvectors (R1), to rtol 1e-10: a small system where every
    kernel is launch-bound, reported as time per solve, per outer and per
    inner iteration, for FP64 and mixed precision with Jacobi and without a
    second level; the oracle's complete solve is the CPU baseline."""
    import torch
    import oracle as O
    from paper_1805_12417_amd import solver as S
    from paper_1805_12417_amd import workloads as W
    w = W.shifted_laplace2d()
    rtol = 1e-10 if args.rtol == 1e-8 else args.rtol
    legs = {}
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)

    def oracle_median(reps=5):
        """median of `reps` complete oracle solves after one warm-up"""
        ro = O.minres_cg(P, O.InnerPC(O.PC_JACOBI, P), w.b, rtol_out=rtol, rtol_in=args.rtol_in)
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            ro = O.minres_cg(P, O.InnerPC(O.PC_JACOBI, P), w.b, rtol_out=rtol,
                             rtol_in=args.rtol_in)
            ts.append(time.perf_counter() - t1)
        return float(np.median(ts)), ro

    cores = O.num_threads()
    t_cpu, ro = oracle_median()
    O.set_num_threads(1)
    t_cpu1, _ = oracle_median()
    O.set_num_threads(cores)
    for prec, pcname in ((S.PREC_FP64, "jacobi"), (S.PREC_MIXED, "jacobi"),
                         (S.PREC_FP64, "none"), (S.PREC_MIXED, "none")):
        key = "%s_%s" % ("mixed" if prec == S.PREC_MIXED else "fp64", pcname)
        s, b = S.from_workload(w, precision=prec)
        pc = s.preconditioner(pcname)
        for _ in range(args.warmup):
            s.solve(b, pc, rtol_out=rtol, rtol_in=args.rtol_in)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            x, st = s.solve(b, pc, rtol_out=rtol, rtol_in=args.rtol_in)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        xg = x.cpu().numpy()
        legs[key] = dict(s_per_solve=round(dt, 5), outer_its=st.outer_its,
                         inner_its=st.inner_its_total, status=st.status_name,
                         us_per_outer_it=round(1e6 * dt / max(1, st.outer_its), 1),
                         us_per_inner_it=round(1e6 * dt / max(1, st.inner_its_total), 2),
                         relres_fp64=float(st.final_relres),
                         x_err_vs_oracle=float(np.linalg.norm(xg - ro["x"]) /
                                               np.linalg.norm(ro["x"])))
        log("laplace2d %s: %.2f ms/solve, %d outer / %d inner its (%.1f us per outer, %.2f us "
            "per inner), relres %.2e, |x - x_oracle|/|x_oracle| %.2e" % (
                key, 1e3 * dt, st.outer_its, st.inner_its_total, 1e6 * dt / max(1, st.outer_its),
                1e6 * dt / max(1, st.inner_its_total), st.final_relres,
                legs[key]["x_err_vs_oracle"]))
        pc.close()
        s.close()
    # the same system as a batch of one in the persistent engine (one launch
    # for the whole solve: no per-kernel launch cost), Jacobi
    dev = torch.device("cuda")
    sysd = (torch.from_numpy(w.row_ptr).to(dev), torch.from_numpy(w.col).to(dev),
            torch.from_numpy(w.val).to(dev),
            torch.from_numpy(np.ascontiguousarray(w.Vhat)).to(dev),
            torch.from_numpy(w.lam).to(dev))
    for prec in (S.PREC_FP64, S.PREC_MIXED):
        key = "%s_jacobi_persistent" % ("mixed" if prec == S.PREC_MIXED else "fp64")
        bs = S.BatchedMinresCG([sysd], 1, precision=prec)
        Bd = [torch.from_numpy(w.b.reshape(1, -1).copy()).to(dev)]
        for _ in range(args.warmup):
            bs.solve(Bd, rtol_out=rtol, rtol_in=args.rtol_in, use_graph=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            X, st, _ = bs.solve(Bd, rtol_out=rtol, rtol_in=args.rtol_in, use_graph=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        xg = X[0][0].cpu().numpy()
        its = int(bs.profile()["team_iters"][0])
        legs[key] = dict(s_per_solve=round(dt, 5), outer_its=int(st.outer_its[0, 0]),
                         inner_its=int(st.inner_its[0, 0]), status=int(st.status[0, 0]),
                         team_blocks=bs.info()[0],
                         us_per_inner_it=round(1e6 * dt / max(1, its), 2),
                         relres_fp64=float(st.relres[0, 0]),
                         x_err_vs_oracle=float(np.linalg.norm(xg - ro["x"]) /
                                               np.linalg.norm(ro["x"])))
        log("laplace2d %s: %.2f ms/solve, %d outer / %d inner its (%.2f us per inner, one "
            "launch of %d blocks), relres %.2e, |x - x_oracle|/|x_oracle| %.2e" % (
                key, 1e3 * dt, st.outer_its[0, 0], st.inner_its[0, 0],
                legs[key]["us_per_inner_it"], legs[key]["team_blocks"], st.relres[0, 0],
                legs[key]["x_err_vs_oracle"]))
        bs.close()
    head = legs["fp64_jacobi"]
    model, ncpu = cpu_info()
    out = {"metric": "time per solve of the 64x64 2D Laplacian (k = 6) to 1e-10",
           "value": head["s_per_solve"], "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * head["s_per_solve"], 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": w.name, "n": w.n, "k": w.k, "rtol_out": rtol,
                      "rtol_in": args.rtol_in, "leg": "fp64_jacobi"},
           "legs": legs,
           "cpu_baseline": {"value": round(t_cpu, 4), "unit": "s", "cores": cores,
                            "kind": "oracle", "cpu_model": model, "nproc": ncpu,
                            "single_thread_s": round(t_cpu1, 4),
                            "sample": "complete FP64 oracle MINRES-CG solve (Jacobi), %d outer / "
                                      "%d inner its; median of 5 after one warm-up, on all "
                                      "threads and on one" % (ro["outer_its"],
                                                               ro["inner_its_total"])}}
    print(json.dumps(out), flush=True)


def N_name(e):
    from paper_1805_12417_amd import _native as N
    return N.STATUS_NAMES.get(e.code, str(e.code))


def bench_learned_eval(args):
    """The learned preconditioner's protocol: one network trained on 16 seeded
    instances of the FE-like family (16^3 nodes x 3 dof, k = 6, seeds
    5000-5015; about 20k pairs in all) for each kind of training pair, then
    evaluated on 8 held-out seeds (5100-5107, 40^3 nodes x 3 dof, k = 15):
    inner iterations and time of the learned + mixed solve next to mixed
    IC-style (incomplete LDL^T(0)) and mixed Jacobi, all to an FP64 true
    relative residual of 1e-8 (the acceptance test of every leg)."""
    import torch
    from paper_1805_12417_amd import learned as LL
    from paper_1805_12417_amd import solver as S
    from paper_1805_12417_amd import workloads as W
    t0 = time.perf_counter()
    fam = [W.shifted_fe27(m=16, k=6, seed=5000 + i, device="cuda") for i in range(16)]
    log("learned eval: 16 training matrices in %.1fs" % (time.perf_counter() - t0))
    per = max(16, args.pairs // 16)
    thetas, train = {}, {}
    for kind in args.pair_kinds.split(","):
        theta, hist, t_train = LL.fit(fam, block_size=3, pairs_per_matrix=per,
                                      steps=args.train_steps, log=log, pairs_kind=kind)
        thetas[kind] = theta
        train[kind] = dict(seconds=round(t_train, 2), loss_first=float(np.mean(hist[:10])),
                           loss_final=float(np.mean(hist[-50:])), pairs=16 * per)
    del fam
    dev = torch.device("cuda")
    rows = []
    for seed in range(5100, 5108):
        w = W.shifted_fe27(m=args.m or 40, k=15, seed=seed, device="cuda")
        row = {"seed": seed, "n": w.n}
        legs = [("learned_" + kd, thetas[kd]) for kd in thetas] + [("ildl0", None),
                                                                   ("jacobi", None)]
        for name, theta in legs:
            s, b = S.from_workload(w, precision=S.PREC_MIXED, autotune=True)
            if theta is not None:
                fac = LL.LearnedFactor(torch.from_numpy(w.row_ptr).to(dev),
                                       torch.from_numpy(w.col).to(dev),
                                       torch.from_numpy(w.val).to(dev), block_size=3,
                                       theta=theta)
                pc = fac.preconditioner(s)
                fac.close()
            else:
                pc = s.preconditioner(name)
            if name == "learned_solver":
                # a network that did not learn can make the inner solves very long:
                # one solve, capped at 20k inner iterations
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                x, st1 = s.solve(b, pc, rtol_out=args.rtol, rtol_in=args.rtol_in,
                                 maxit_inner_total=20000)
                torch.cuda.synchronize()
                dt, st = time.perf_counter() - t1, [st1]
            else:
                dt, x, st = time_solves(s, pc, b, max(1, args.steps), 1, args.rtol, args.rtol_in)
            rel = float(torch.linalg.vector_norm(b - s.spmv(x)) / torch.linalg.vector_norm(b))
            row[name] = dict(inner_its=st[-1].inner_its_total, outer_its=st[-1].outer_its,
                             seconds=round(dt, 4), relres_fp64=rel, status=st[-1].status_name)
            log("seed %d %s: %s inner %d, %.3f s" % (seed, name, st[-1].status_name,
                                                    st[-1].inner_its_total, dt))
            pc.close()
            s.close()
        log("seed %d: %s" % (seed, {k: (v["inner_its"], v["seconds"]) for k, v in row.items()
                                    if isinstance(v, dict)}))
        rows.append(row)
    names = [k for k in rows[0] if isinstance(rows[0][k], dict)]
    mean = {k: dict(inner_its=float(np.mean([r[k]["inner_its"] for r in rows])),
                    seconds=float(np.mean([r[k]["seconds"] for r in rows])),
                    converged=sum(r[k]["status"] == "OK" for r in rows)) for k in names}
    print(json.dumps({"workload": "learned_eval_fe27_40^3x3_k15", "train": train,
                      "held_out": rows, "mean": mean,
                      "note": "learned_solver legs are capped at 20k inner iterations"}),
          flush=True)


BATCH_K_BUCKETS = (8, 16, 32, 40, 48, 64)


def batched_iter_bytes(w, nr, elem):
    """Model bytes of one inner CG iteration of a persistent-launch team
    (FP32 or FP64 inner, nr right-hand sides interleaved): the CSR matrix
    once (values and columns, row pointers), the rows of Vhat once (plus the
    refresh every 32nd iteration), the nr-wide vectors p (gathered once), q,
    then z, r, p, q read and z, r written, then r, p read and p written (11
    accesses), and 1/diag(A) in each of the three phases."""
    n, nnz, k = w.n, w.nnz, w.k
    return (nnz * (elem + 4) + 4 * (n + 1) + n * k * elem * (1 + 1 / 32) + 11 * n * nr * elem
            + 3 * n * elem)


def batched_roofline(bs, ws, teams):
    """Per persistent launch (k bucket): the wall-clock span of its teams,
    the fraction of block-time its teams were busy, and the model bytes of
    the inner iterations the teams ran divided by the span (outer MINRES
    work, a few percent, not counted)."""
    prof = bs.profile()
    nr = 8
    out = []
    for g in sorted(set(prof["group"].tolist())):
        mem = [i for i in range(len(ws)) if prof["group"][i] == g]
        t0 = min(prof["t_begin"][i] for i in mem)
        t1 = max(prof["t_end"][i] for i in mem)
        span = t1 - t0
        blocks = sum(teams[i] for i in mem)
        busy = sum(teams[i] * (prof["t_end"][i] - prof["t_begin"][i]) for i in mem)
        model = sum(batched_iter_bytes(ws[i], nr, 4) * int(prof["team_iters"][i]) for i in mem)
        kb = next(b for b in BATCH_K_BUCKETS if b >= max(1, max(ws[i].k for i in mem)))
        # phase split of the team that ran longest (its first workgroup's clock)
        slow = max(mem, key=lambda i: prof["t_end"][i] - prof["t_begin"][i])
        ph = prof["phase_s"][slow]
        its = max(1, int(prof["team_iters"][slow]))
        split = {name: round(1e6 * ph[q] / its, 2) for q, name in enumerate(
            ("A_work_us", "A_reduce_us", "B_work_us", "B_reduce_us", "C_work_us", "C_sync_us"))}
        split.update(n=ws[slow].n, k=ws[slow].k, team=teams[slow],
                     model_GBps=round(batched_iter_bytes(ws[slow], nr, 4) * its /
                                      max(1e-12, prof["t_end"][slow] - prof["t_begin"][slow]) / 1e9, 1))
        per_sys = [{"n": ws[i].n, "k": ws[i].k, "team": teams[i],
                    "team_iters": int(prof["team_iters"][i]),
                    "s": round(float(prof["t_end"][i] - prof["t_begin"][i]), 4)} for i in mem]
        out.append({"launch": g, "k_bucket": kb, "systems": len(mem), "blocks": blocks,
                    "per_system": per_sys,
                    "slowest_team_per_iteration": split,
                    "span_s": round(span, 4), "busy_frac": round(busy / (blocks * span), 3),
                    "team_iters_max": int(max(prof["team_iters"][i] for i in mem)),
                    "model_bytes": float(model), "achieved_TBps": round(model / span / 1e12, 3),
                    "frac_of_peak": round(model / span / 8e12, 3)})
    return out


def bench_batched(args):
    """48 shifted systems of uneven size (n log-uniform in [2e4, 5e5]), 8
    right-hand sides each (FP32 inner / FP64 outer, Jacobi), in both batched
    modes: one persistent launch per k bucket replayed from a HIP graph
    (teams re-planned at setup from a calibration solve with other
    right-hand sides), and the single-system kernels on several concurrent
    streams.  A sample of systems
    is also solved one right-hand side at a time on one stream, for
    comparison."""
    import torch
    from paper_1805_12417_amd import solver as S
    from paper_1805_12417_amd import workloads as W
    t0 = time.perf_counter()
    sizes = W.batch_sizes(count=args.nsys)
    ws = []
    for i, (d, k) in enumerate(sizes):
        ws.append(W.shifted_laplace3d(seed=4000 + i, dims=d, k=k, device="cuda"))
        log("system %d/%d: n=%d k=%d (%.1fs)" % (i + 1, len(sizes), ws[-1].n, k,
                                                time.perf_counter() - t0))
    log("batched: %d systems, n %d..%d (sum %d), setup %.1fs" % (
        len(ws), min(w.n for w in ws), max(w.n for w in ws), sum(w.n for w in ws),
        time.perf_counter() - t0))
    dev = torch.device("cuda")
    systems = [(torch.from_numpy(w.row_ptr).to(dev), torch.from_numpy(w.col).to(dev),
                torch.from_numpy(w.val).to(dev),
                torch.from_numpy(np.ascontiguousarray(w.Vhat)).to(dev),
                torch.from_numpy(w.lam).to(dev)) for w in ws]
    rng = np.random.default_rng(4999)
    Bs = [torch.from_numpy(rng.standard_normal((8, w.n))).to(dev) for w in ws]
    bs = S.BatchedMinresCG(systems, 8, precision=S.PREC_MIXED)
    nb, teams = bs.info()

    def worst_relres(X):
        # FP64 true residuals recomputed with each system's FP64 SpMV
        worst = 0.0
        for i, w in enumerate(ws):
            s1 = S.MinresCG(*systems[i], precision=S.PREC_FP64)
            for j in range(8):
                r = Bs[i][j] - s1.spmv(X[i][j].contiguous())
                worst = max(worst, float(torch.linalg.vector_norm(r) /
                                         torch.linalg.vector_norm(Bs[i][j])))
            s1.close()
        return worst

    modes = {}
    for mode in args.batch_modes.split(","):
        kw = dict(rtol_out=args.rtol, rtol_in=args.rtol_in)
        if mode == "persistent":
            kw["use_graph"] = True
            # setup: teams sized by each system's inner iterations, taken from
            # one solve with other right-hand sides (the same systems solved
            # again and again, as in shift-and-invert)
            rng_cal = np.random.default_rng(4998)
            Bcal = [torch.from_numpy(rng_cal.standard_normal((8, w.n))).to(dev) for w in ws]
            _, stc, _ = bs.solve(Bcal, rtol_out=args.rtol, rtol_in=args.rtol_in)
            # the iterations each team ran (it iterates while any of its
            # right-hand sides is active)
            bs.rebalance(np.maximum(1, bs.profile()["team_iters"]))
            for r in range(args.measured_rebalance):
                # further calibration solves (other right-hand sides again);
                # the teams then re-planned by the block-time each system took
                rng_cal = np.random.default_rng(4996 - r)
                Bcal = [torch.from_numpy(rng_cal.standard_normal((8, w.n))).to(dev) for w in ws]
                bs.solve(Bcal, rtol_out=args.rtol, rtol_in=args.rtol_in)
                bs.rebalance_measured()
            del Bcal
            nb, teams = bs.info()
            log("batched persistent: teams re-planned from %d calibration solves" % (
                1 + args.measured_rebalance))
        elif mode.startswith("streams"):
            kw["streams"] = int(mode[len("streams"):] or 4)
        else:
            raise SystemExit("unknown batch mode %r" % mode)
        for _ in range(args.warmup):
            bs.solve(Bs, **kw)
            log("batched %s: warmup step done" % mode)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            X, st, rc = bs.solve(Bs, **kw)
            log("batched %s: timed step done" % mode)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        worst = worst_relres(X)
        log("batched %s: %.3f s for %d systems x 8 rhs, worst relres %.2e, status max %d" % (
            mode, dt, len(ws), worst, int(st.status.max())))
        modes[mode] = {"s": round(dt, 4), "worst_relres_fp64": worst,
                       "max_status": int(st.status.max()),
                       "outer_its_max": int(st.outer_its.max()),
                       "inner_its_max": int(st.inner_its.max())}
        if mode == "persistent":
            modes[mode]["launches"] = batched_roofline(bs, ws, teams)
            for g in modes[mode]["launches"]:
                log("batched persistent launch %d (k <= %d, %d systems, %d blocks): %.3f s, "
                    "team busy %.0f%%, model %.1f GB -> %.2f TB/s (%.2f of peak)" % (
                        g["launch"], g["k_bucket"], g["systems"], g["blocks"], g["span_s"],
                        100 * g["busy_frac"], g["model_bytes"] / 1e9, g["achieved_TBps"],
                        g["frac_of_peak"]))
                log("  slowest team per iteration: %s" % g["slowest_team_per_iteration"])
    # unbatched reference on a sample of systems: one rhs at a time, one stream
    sample = [] if args.no_unbatched else list(range(0, len(ws), max(1, len(ws) // 6)))
    t_unb = 0.0
    for i in sample:
        s1 = S.MinresCG(*systems[i], precision=S.PREC_MIXED)
        pc = s1.preconditioner("jacobi")
        s1.solve(Bs[i][0].contiguous(), pc, rtol_out=args.rtol, rtol_in=args.rtol_in)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for j in range(8):
            s1.solve(Bs[i][j].contiguous(), pc, rtol_out=args.rtol, rtol_in=args.rtol_in)
        torch.cuda.synchronize()
        t_unb += time.perf_counter() - t2
        s1.close()
    est_unb = t_unb * len(ws) / len(sample) if sample else float("nan")
    best = min(modes, key=lambda m: modes[m]["s"])
    dt = modes[best]["s"]
    out = {"metric": "time to solve 48 shifted systems x 8 rhs to 1e-8 FP64 relative residual",
           "value": dt, "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * dt, 1), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 inner / f64 outer",
           "data": "synthetic",
           "config": {"workload": "batched_shifted_laplace3d", "systems": len(ws),
                      "sum_n": sum(w.n for w in ws), "nrhs": 8, "rtol_out": args.rtol,
                      "rtol_in": args.rtol_in, "mode": best, "persistent_blocks": nb},
           "modes": modes,
           "unbatched_estimate_s": round(est_unb, 3) if sample else None,
           "unbatched_sample": "%d of %d systems solved one rhs at a time with the single-system "
                               "solver on one stream, scaled by the system count" % (
                                   len(sample), len(ws)),
           "speedup_vs_unbatched": round(est_unb / dt, 2) if sample else None}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fe27",
                    help="fe27 (default), laplace3d, batched, brake, learned-eval, kkt, "
                         "laplace2d")
    ap.add_argument("--m", type=int, default=0, help="grid size override (testing)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--rtol-in", type=float, default=1e-4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-steps", type=int, default=2000,
                    help="Adam steps of the learned factor's training (setup, untimed)")
    ap.add_argument("--cpu-budget", type=float, default=30.0,
                    help="at most about this many seconds of oracle work in the CPU baseline")
    ap.add_argument("--oracle-x", action="store_true",
                    help="fe27: a full oracle solve for the per-leg errors even when the CPU "
                         "baseline's solve was capped")
    ap.add_argument("--pairs", type=int, default=20480,
                    help="learned-eval: training pairs over the 16 training matrices")
    ap.add_argument("--pair-kinds", default="mx,solver",
                    help="learned-eval: kinds of training pairs to compare")
    ap.add_argument("--legs", default="",
                    help="fe27, kkt: comma list of legs to run (e.g. mixed_learned), for "
                         "profiling; fe27 then prints the legs and the roofline only")
    ap.add_argument("--no-laplace-spmv", action="store_true",
                    help="fe27: skip the 128^3 Laplacian SpMV rates")
    ap.add_argument("--no-eigs", action="store_true", help="skip the GPU setup-stage timing")
    ap.add_argument("--nsys", type=int, default=48, help="batched: number of systems")
    ap.add_argument("--no-unbatched", action="store_true",
                    help="batched: skip the one-rhs-at-a-time comparison (for profiling)")
    ap.add_argument("--measured-rebalance", type=int, default=1,
                    help="batched: calibration solves after the first, each followed by teams "
                         "re-planned from the block-time each system took (0: iteration "
                         "counts only)")
    ap.add_argument("--batch-modes", default="streams8,persistent",
                    help="batched: comma list of persistent, streamsS (S concurrent streams)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 20 plain device copies of MIB MiB (calibrates the HBM "
                         "byte counters of a profiler against a known traffic)")
    ap.add_argument("--mmr-form", type=int, default=0,
                    help="0: autotuned, 1: fused M_mr kernel, 2: SpMV + rank-k pass")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_12417_amd import solver as S
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(20):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                          "launches": 20}), flush=True)
        return
    if args.workload == "fe27":
        return bench_fe27(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "brake":
        return bench_brake(args)
    if args.workload == "learned-eval":
        return bench_learned_eval(args)
    if args.workload == "kkt":
        return bench_kkt(args)
    if args.workload == "laplace2d":
        return bench_laplace2d(args)
    return bench_laplace3d(args)


def bench_laplace3d(args):
    """128^3 7-point random-coefficient Laplacian, k = 20: mixed Jacobi,
    learned + mixed (trained on 40^3 matrices of the family), MINRES-CG*,
    plain FP64; roofline of the Jacobi iteration's update kernel."""
    import torch
    from paper_1805_12417_amd import solver as S
    t0 = time.perf_counter()
    w = make_workload(args.workload, args.m, "cuda")
    log("workload %s n=%d nnz=%d k=%d setup %.1fs" % (w.name, w.n, w.nnz, w.k,
                                                     time.perf_counter() - t0))
    # solves are timed on handles without per-launch events; the roofline
    # kernel is timed by HIP events around each of its launches in a second
    # timed region (the same mixed Jacobi solves on a profiling handle)
    sm, b = S.from_workload(w, precision=S.PREC_MIXED, autotune=True, mmr_form=args.mmr_form)
    pcm = sm.preconditioner("jacobi")
    dt_m, xm, stm = time_solves(sm, pcm, b, args.steps, args.warmup, args.rtol, args.rtol_in)
    sprof, _ = S.from_workload(w, precision=S.PREC_MIXED, profile=True, autotune=True,
                               mmr_form=args.mmr_form)
    pcprof = sprof.preconditioner("jacobi")
    dt_prof, _, _ = time_solves(sprof, pcprof, b, args.steps, args.warmup, args.rtol, args.rtol_in)
    kms, klaunch = sprof.kernel_time()
    pcprof.close()
    sprof.close()
    log("mixed: %.3f s/solve (%.3f s with per-launch events) status=%s outer=%d inner=%d "
        "relres=%.2e lanes=%d split=%d mmr %.1f us" % (
            dt_m, dt_prof, stm[-1].status_name, stm[-1].outer_its, stm[-1].inner_its_total,
            stm[-1].final_relres, sm.lanes, sm.mmr_split, kms / max(klaunch, 1) * 1e3))
    # FP64 true residual of the returned x, recomputed by the library's FP64 SpMV
    r = b - sm.spmv(xm)
    relres_m = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))

    # learned + mixed: C C^T from the network (trained on smaller matrices of
    # the same family), FP32 inner CG, FP64 outer MINRES
    learned = None
    if not args.no_learned:
        from paper_1805_12417_amd import learned as LL
        from paper_1805_12417_amd import workloads as W
        t1 = time.perf_counter()
        fam = [W.shifted_laplace3d(seed=1000 + i, m=40, k=w.k, device="cuda") for i in range(4)]
        log("learned: %d training matrices (40^3) in %.1fs" % (len(fam), time.perf_counter() - t1))
        theta, hist, t_train = LL.fit(fam, block_size=1, steps=args.train_steps, log=log)
        dev = torch.device("cuda")
        fac = LL.LearnedFactor(torch.from_numpy(w.row_ptr).to(dev), torch.from_numpy(w.col).to(dev),
                               torch.from_numpy(w.val).to(dev), block_size=1, theta=theta)
        t1 = time.perf_counter()
        pcl = fac.preconditioner(sm)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t1
        dt_l, xl, stl = time_solves(sm, pcl, b, args.steps, args.warmup, args.rtol, args.rtol_in)
        rl = b - sm.spmv(xl)
        relres_l = float(torch.linalg.vector_norm(rl) / torch.linalg.vector_norm(b))
        log("learned+mixed: %.3f s/solve status=%s outer=%d inner=%d relres=%.2e "
            "(inference + C^T build %.3fs, network forward %.2f ms)" % (
                dt_l, stl[-1].status_name, stl[-1].outer_its, stl[-1].inner_its_total, relres_l,
                t_inf, fac.forward_ms()))
        learned = dict(seconds=round(dt_l, 5), outer_its=stl[-1].outer_its,
                       inner_its_total=stl[-1].inner_its_total, final_relres_fp64=relres_l,
                       status=stl[-1].status_name, train_s=round(t_train, 2),
                       train_loss_final=float(np.mean(hist[-50:])),
                       setup_s=round(t_inf, 3), network_forward_ms=round(fac.forward_ms(), 3),
                       train_matrices="4 x shifted laplace3d 40^3, seeds 1000-1003")
        fac.close()

    # MINRES-CG* (the SMW-improved second level, Jacobi-based), mixed precision
    pcs = sm.preconditioner("jacobi", smw=True)
    dt_s, xs, sts = time_solves(sm, pcs, b, args.steps, args.warmup, args.rtol, args.rtol_in)
    rs = b - sm.spmv(xs)
    smw = dict(seconds=round(dt_s, 5), outer_its=sts[-1].outer_its,
               inner_its_total=sts[-1].inner_its_total,
               final_relres_fp64=float(torch.linalg.vector_norm(rs) / torch.linalg.vector_norm(b)),
               status=sts[-1].status_name)
    log("mixed MINRES-CG* (Jacobi + SMW term): %.3f s/solve status=%s outer=%d inner=%d" % (
        dt_s, sts[-1].status_name, sts[-1].outer_its, sts[-1].inner_its_total))
    pcs.close()

    plain = None
    if not args.no_plain:
        sp, _ = S.from_workload(w, precision=S.PREC_FP64, autotune=True, mmr_form=args.mmr_form)
        pcp = sp.preconditioner("jacobi")
        dt_p, xp, stp = time_solves(sp, pcp, b, args.steps, args.warmup, args.rtol, args.rtol_in)
        log("fp64 : %.3f s/solve status=%s outer=%d inner=%d relres=%.2e" % (
            dt_p, stp[-1].status_name, stp[-1].outer_its, stp[-1].inner_its_total,
            stp[-1].final_relres))
        spmv64_ms = time_spmv(sp, 0, w)
        plain = dict(seconds=dt_p, outer_its=stp[-1].outer_its,
                     inner_its_total=stp[-1].inner_its_total, final_relres=stp[-1].final_relres,
                     status=stp[-1].status_name)
    spmv32_ms = time_spmv(sm, 1, w)

    avg_ms = kms / max(klaunch, 1)
    bytes_k = mmr_bytes(w, 4, sm.block_csr, sm.sliced_ell)
    if (sm.sliced_ell or sm.block_csr) and sm.mmr_split and w.k > 0:
        # the iteration's dominant kernel: the CG update that streams Vhat and
        # forms q = Ap + Vhat (c o s) (A p comes from the sliced SpMV before it)
        form = "update_v"
        kname = ("k_cg_update_v<float, KB, true>: rank-k part of the M_mr apply fused with the "
                 "Jacobi CG update (Vhat, z, r read and written, p, Ap, D^-1 read)")
        bytes_k = w.n * w.k * 4 + 7 * w.n * 4
        model = "4nk (Vhat) + 7 x 4n (z, r read and written; p, Ap, D^-1 read)"
    elif sm.sliced_ell:
        form, kname = "sell", ("M_mr apply, fp32: k_sell_mmr (sliced ELL, %d-bit columns, one "
                               "pass)" % sm.sliced_ell)
    elif sm.mmr_split:
        form, kname = "split", "M_mr apply, fp32: k_spmv_chk + k_mmr_vpart (split)"
    else:
        form, kname = "fused", "M_mr apply, fp32: k_mmr (SpMV + Vhat(c*s) fused)"
    if form != "update_v":
        model = "A in its storage (values, columns, pointers) + 2 x 4n (p, q) + 4nk (Vhat)"
    achieved = bytes_k / (avg_ms * 1e-3) / 1e9
    roofline = dict(bound="hbm", kernel=kname,
                    achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 4),
                    traffic=MMR_TRAFFIC_BYTES.get((w.name, form)),
                    avg_launch_us=round(avg_ms * 1e3, 2), launches=klaunch,
                    algorithmic_bytes=bytes_k, bytes_model=model)
    spmv = dict(fp32_us=round(spmv32_ms * 1e3, 2),
                fp32_GBps=round(spmv_bytes(w, 4, sm.block_csr, sm.sliced_ell) /
                                (spmv32_ms * 1e-3) / 1e9, 1))
    if plain:
        spmv.update(fp64_us=round(spmv64_ms * 1e3, 2),
                    fp64_GBps=round(spmv_bytes(w, 8, sp.block_csr, sp.sliced_ell) /
                                    (spmv64_ms * 1e-3) / 1e9, 1))

    # setup stage on the GPU: the k smallest eigenpairs (V-hat, Lambda-hat),
    # compared with the input generator's (an independent implementation)
    deflation = None
    if not args.no_eigs:
        dev = torch.device("cuda")
        rp_d, ci_d, va_d = (torch.from_numpy(a).to(dev) for a in (w.row_ptr, w.col, w.val))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lam_g, V_g, est = S.lowest_eigs(rp_d, ci_d, va_d, w.k, tol=1e-10)
        torch.cuda.synchronize()
        t_eig = time.perf_counter() - t1
        deflation = dict(seconds=round(t_eig, 3), outer_its=est["outer_its"],
                         block_products=est["spmm_calls"], converged=bool(est["converged"]),
                         max_residual_rel=est["max_residual"] / est["bound"],
                         max_abs_lam_diff_vs_input=float(np.abs(lam_g - w.lam).max()),
                         negative=est["negative"], method="Chebyshev-filtered subspace iteration, "
                         "FP64, tol 1e-10 x Gershgorin bound")
        log("deflation setup (k = %d smallest eigenpairs): %.2fs, %d outer, converged %s, "
            "max |lam - lam_input| %.2e" % (w.k, t_eig, est["outer_its"], bool(est["converged"]),
                                            deflation["max_abs_lam_diff_vs_input"]))
        del V_g, rp_d, ci_d, va_d

    cpu = None
    if not args.no_cpu:
        ref = plain if plain else dict(inner_its_total=stm[-1].inner_its_total,
                                       outer_its=stm[-1].outer_its)
        cpu, _ = cpu_baseline(w, ref["inner_its_total"], ref["outer_its"], args.rtol, args.rtol_in,
                           args.cpu_budget)
        log("cpu baseline: %.2f s (estimated), %d threads" % (cpu["value"], cpu["cores"]))

    mixed_jacobi = dict(seconds=round(dt_m, 5), outer_its=stm[-1].outer_its,
                        inner_its_total=stm[-1].inner_its_total, final_relres_fp64=relres_m,
                        status=stm[-1].status_name)
    head = learned if learned else mixed_jacobi
    dt_h = head["seconds"]
    out = {
        "metric": ("time-to-1e-8 FP64 relative residual, learned+mixed MINRES-CG vs plain FP64"
                   if learned else
                   "time-to-1e-8 FP64 relative residual, MINRES-CG FP32-inner/FP64-outer (Jacobi)"),
        "value": round(dt_h, 5), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt_h * 1e3, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 inner / f64 outer",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nnz": w.nnz, "k": w.k, "rtol_out": args.rtol,
                   "rtol_in": args.rtol_in,
                   "precond": "learned C C^T" if learned else "jacobi", "parallelism": "none",
                   "spmv_lanes": sm.lanes, "mmr_split": sm.mmr_split,
                   "a_format": ("sliced_ell%d" % sm.sliced_ell if sm.sliced_ell else
                                "bsr%d" % sm.block_csr if sm.block_csr else "csr")},
        "outer_its": head["outer_its"], "inner_its_total": head["inner_its_total"],
        "final_relres_fp64": head["final_relres_fp64"], "status": head["status"],
        "learned_mixed": learned,
        "mixed_jacobi": mixed_jacobi,
        "mixed_minres_cg_star": smw,
        "plain_fp64": plain,
        "speedup_vs_plain_fp64": round(plain["seconds"] / dt_h, 3) if plain else None,
        "spmv": spmv,
        "roofline": roofline,
        "deflation_setup_gpu": deflation,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
