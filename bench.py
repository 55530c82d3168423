"""Benchmark of the multi-period AC OPF evaluation sweep on one MI355X.

A step is one whole per-iteration evaluation sweep (objective, gradient,
constraints, Jacobian, Hessian, J^T v and the condensed KKT matrix) of the
paper-scale synthetic instance (N=10000 buses, B=13000 lines, G=2000
generators, T=168 periods: 12.77M variables), inputs resident in HBM, one
replay of the sweep's HIP graph per step.  value = (nnz J + nnz H + nnz K)
per step / step time.  The same steps are also run eagerly with every
kernel timed by HIP events (the roofline of the dominant kernel).  The same run times
the batched form (64 uneven instances, one graph replay vs 64 plain sweeps)
and the adjoint form (16 mid instances, matrix-free vs per-instance
Jacobian + COO product), and the CPU oracle on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Jac+Hess+KKT nnz/s and HBM GB/s at 12.7M vars; batched & adjoint vs plain"
TUNE_CACHE = os.path.join(ROOT, "paper_2405_14032_amd", "tune", "mi355x.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def call_bytes(net, model):
    """Algorithmic bytes per call (8-byte values moved at least once)."""
    N, B, G, T = net.N, net.B, net.G, net.T
    n, m, nj, nh, nk = model.n, model.m, model.nnz_jac, model.nnz_hess, model.nnz_kkt
    return {
        "obj": 8 * (G * T),
        "grad": 8 * (n + G * T),
        "cons": 8 * (m + n + 2 * N * T),
        "jac": 8 * (nj + 2 * N * T + 4 * B * T),
        "hess": 8 * (nh + 2 * N * T + 6 * B * T + G),
        "jtprod": 8 * (2 * n + m),
        "condensed": 8 * (nj + nh + m + n + nk),
        # fused J + H + K: x (vm, va, flows), 6 multipliers per line-period,
        # c2, row weights, diagonal in; J, H, K out
        "jhk": 8 * (2 * N * T + 4 * B * T + 6 * B * T + G + m + n + nj + nh + nk),
        # lifted-KKT calls: x (vm, va, flows) and v in, J v out
        "jprod": 8 * (2 * N * T + 4 * B * T + n + m),
        # x, its bounds and multipliers, grad; s, y, slack bounds and
        # multipliers, c; diag_x, dcon, rhs out
        "condensed_rhs": 8 * (8 * n + 8 * m),
        # the same state and dx in; ds, dy, dvl, dvu, dzl, dzu out
        "recover_step": 8 * (8 * n + 11 * m),
    }


def sweep_kernel_bytes(net, model, kbus):
    """Algorithmic bytes of the whole sweep and of its two fused kernels
    (8-byte values each kernel must read or write at least once; the
    line-to-bus hand-off records and index tables are not counted)."""
    N, B, G, T = net.N, net.B, net.G, net.T
    n, m, nj, nh, nk = model.n, model.m, model.nnz_jac, model.nnz_hess, model.nnz_kkt
    NT, BT, GT, G1 = N * T, B * T, G * T, G * (T - 1)
    sweep_a = (2 * NT + 4 * BT + GT          # x: vm, va, flows, pg
               + 6 * BT                      # lambda: flow and thermal rows
               + 7 * BT + 2 * NT + G1        # v: line rows, balance rows, ramp rows
               + 7 * BT + 2 * NT + G1        # d: the same rows
               + 4 * BT + 2 * GT             # diag_x: flow and generator variables
               + nj + nh + (nk - kbus)       # J, H, K line / generator rows
               + 7 * BT + G1                 # c: line and ramp rows
               + 4 * BT + 2 * GT             # J^T v: flow and generator variables
               + 4 * BT + 2 * GT)            # gradient: same
    sweep_b = (4 * BT + 2 * GT + T           # x: flows, pg, qg, reference angle
               + 2 * NT                      # load profile
               + 2 * NT + 3 * T              # diag_x (vm, va); v, d, J of the reference row
               + kbus                        # K bus rows
               + 2 * NT + T                  # c: balance and reference rows
               + 2 * NT + 2 * NT)            # J^T v and gradient on vm, va
    sweep = (n + 6 * BT + m + m + n + 2 * NT + n + m + nj + nh + nk + n + model.ninst)
    return {"sweep_a": 8 * sweep_a, "sweep_b": 8 * sweep_b, "sweep": 8 * sweep}


def event_time(torch, fn, reps):
    """Median milliseconds of fn() over reps (one warm-up first), a HIP event
    pair per repetition on the current stream."""
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    fn()
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(s)
        fn()
        e1.record(s)
    ev[-1][1].synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))


def copy_peak(torch, dev, reps=5):
    """Measured HBM rate of a plain 1 GiB device-to-device copy (1 GiB read
    + 1 GiB written per copy), median of ``reps`` after a warm-up: the
    practical peak next to the 8 TB/s of the data sheet."""
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    ms = event_time(torch, lambda: dst.copy_(src), reps)
    nbytes = 2 * src.numel() * 8
    del src, dst
    return {"bytes_per_copy": nbytes, "ms": round(ms, 4), "gbs": round(nbytes / ms / 1e6, 1)}


PROFILE = os.path.join(ROOT, "profiles", "sweep_paper_scale.txt")
KERNEL_SOURCES = ("paper_2405_14032_amd/csrc/opf_kernels.hip", "paper_2405_14032_amd/csrc/opf_device.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3
    summary (calibrated FETCH_SIZE + WRITE_SIZE), or None when the summary
    is missing or was taken on other kernel sources."""
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    m = re.search(r"kernel sources sha256\[:16\][^:]*:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    for line in text.splitlines():
        f = line.split()
        if f and f[0] == kernel and len(f) == 9:
            return float(f[8]) * 1e6
    return None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_chunk_worker(chunk, periods, conn):
    """One worker of the CPU baseline: builds its share of the paper-scale
    horizon once, then runs one whole oracle sweep per request and reports
    the J + H + K nnz it produced."""
    from oracle import opf_oracle as O
    from paper_2405_14032_amd import synth
    t0, t1 = chunk
    full = synth.make_network(10000, 13000, 2000, periods, 3)
    net = synth.make_network(10000, 13000, 2000, t1 - t0, 3)
    net.pd, net.qd = full.pd[t0:t1].copy(), full.qd[t0:t1].copy()
    pt = synth.make_point(net, 3 + t0)
    L = O.Layout(net)
    conn.send("ready")
    while conn.recv() == "run":
        O.objective(net, pt.x)
        O.gradient(net, pt.x)
        O.constraints(net, pt.x)
        jac = O.jacobian(net, pt.x)
        hess = O.hessian(net, pt.x, pt.lam, pt.sigma)
        O.jtprod(net, pt.x, pt.lam)
        rp, _, _, _ = O.condensed(L.n, jac, hess, pt.diag_x, pt.dcon)
        conn.send(len(jac[0]) + len(hess[0]) + int(rp[-1]))


def cpu_baseline(periods: int = 96, reps: int = 5, max_workers: int = 16):
    """The oracle as it stands, timed on the host cores: the paper-scale grid
    over a horizon of ``periods`` (a bounded sample) split into one
    contiguous period range per worker process (each range its own horizon,
    so the ramp rows at the range boundaries are the only thing missing),
    all workers sweeping at once; one warm-up, then the median wall time of
    ``reps`` sweeps; nnz/s like the GPU value.  Call it before anything
    initialises the GPU: the workers are fresh interpreters (spawn)."""
    import multiprocessing as mp
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(max_workers, avail, periods))
    bounds = [round(k * periods / workers) for k in range(workers + 1)]
    ctx = mp.get_context("spawn")
    procs, conns = [], []
    # one thread per worker: the workers inherit this environment
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    os.environ.update({k: "1" for k in saved})
    try:
        for k in range(workers):
            a, b = ctx.Pipe()
            p = ctx.Process(target=_oracle_chunk_worker, args=((bounds[k], bounds[k + 1]), periods, b), daemon=True)
            p.start()
            procs.append(p)
            conns.append(a)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    for c in conns:
        assert c.recv() == "ready"
    times, nnz = [], 0
    for r in range(reps + 1):
        t0 = time.perf_counter()
        for c in conns:
            c.send("run")
        nnz = sum(c.recv() for c in conns)
        dt = time.perf_counter() - t0
        if r > 0:
            times.append(dt)
    for c in conns:
        c.send("stop")
    for p in procs:
        p.join(timeout=30)
    med = float(np.median(times))
    return {"value": nnz / med, "unit": "nnz/s", "cores": workers, "kind": "oracle",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "affinity_cpus": avail,
            "median_s": round(med, 3), "times_s": [round(t, 3) for t in times],
            "sample": f"one full sweep (f, grad, c, J, H, J^T v, K) of the paper-scale grid (N=10000, B=13000, "
                      f"G=2000) over T={periods} periods, split into {workers} contiguous period ranges swept "
                      f"at once by {workers} worker processes (numpy/scipy, one thread each): {nnz} J+H+K nnz; "
                      f"median of {reps} after one warm-up"}


def make_inputs(torch, dev, net, pt):
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    return t(pt.x), t(pt.lam), t(pt.diag_x), t(pt.dcon)


def outputs(torch, dev, model):
    e = lambda k: torch.empty(k, dtype=torch.float64, device=dev)
    return dict(f=e(model.ninst), grad=e(model.n), c=e(model.m), jvals=e(model.nnz_jac),
                hvals=e(model.nnz_hess), jtv=e(model.n), kvals=e(model.nnz_kkt))


def bench_plain(torch, dev, args):
    from paper_2405_14032_amd import capi, synth
    net = synth.config_network("paper")
    pt = synth.make_point(net, 3)
    log(f"paper-scale instance: N={net.N} B={net.B} G={net.G} T={net.T}")
    torch.cuda.synchronize()
    t_create = time.perf_counter()
    M = capi.Model([net], device=0)  # host symbolic analysis + upload (once per model)
    create_s = time.perf_counter() - t_create
    M.use_current_torch_stream()
    M.autotune(args.tune_cache)
    X, LAM, DX, D = make_inputs(torch, dev, net, pt)
    out = outputs(torch, dev, M)
    sa = M.sweep_args(x=X, lam=LAM, sigma=pt.sigma, v=LAM, diag_x=DX, dcon=D, **out)
    # the timed steps: the whole sweep recorded once into a HIP graph and
    # replayed, one graph launch per step (how an interior-point loop calls it)
    for _ in range(args.warmup):
        M.sweep_graph(sa)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        M.sweep_graph(sa)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    # the same replays one by one between HIP events: the median step
    median_step_ms = event_time(torch, lambda: M.sweep_graph(sa), args.steps)
    # the same steps launched eagerly, every kernel bracketed by HIP events on
    # the model's stream: the per-kernel durations of the roofline (median
    # over the steps, one launch of each kernel per step)
    for _ in range(args.warmup):
        M.sweep(sa)
    torch.cuda.synchronize()
    per_kernel = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        M.set_timing(True)
        M.sweep(sa)
        for k, (c, t) in M.kernel_stats().items():
            per_kernel.setdefault(k, []).append(t / c)
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    M.set_timing(False)
    kernels = {k: {"launches": len(v), "median_ms": round(float(np.median(v)), 4),
                   "mean_ms": round(float(np.mean(v)), 4)} for k, v in per_kernel.items()}
    nnz = M.nnz_jac + M.nnz_hess + M.nnz_kkt
    by = call_bytes(net, M)
    # K slots in the bus (vm, va) rows: written by the bus pass of the sweep
    rp = torch.empty(M.n + 1, dtype=torch.int64, device=dev)
    ci = torch.empty(M.nnz_kkt, dtype=torch.int32, device=dev)
    M.kkt_structure(rp, ci)
    n_p = 2 * net.N + 2 * net.G + 4 * net.B
    starts = torch.arange(net.T, device=dev) * n_p
    kbus = int((rp[starts + 2 * net.N] - rp[starts]).sum())
    # symbolic outputs (J / H COO indices, K CSR) generated on the device
    jr, jc = (torch.empty(M.nnz_jac, dtype=torch.int32, device=dev) for _ in range(2))
    hr, hc = (torch.empty(M.nnz_hess, dtype=torch.int32, device=dev) for _ in range(2))
    symbolic = {"model_create_s": round(create_s, 3),
                "jac_structure_ms": round(event_time(torch, lambda: M.jac_structure(jr, jc), 3), 4),
                "hess_structure_ms": round(event_time(torch, lambda: M.hess_structure(hr, hc), 3), 4),
                "kkt_structure_ms": round(event_time(torch, lambda: M.kkt_structure(rp, ci), 3), 4)}
    del jr, jc, hr, hc, ci
    kb = sweep_kernel_bytes(net, M, kbus)
    # per-call times, events on the model's (current) stream
    calls = {
        "obj": lambda: M.eval_obj(X, out["f"]),
        "grad": lambda: M.eval_grad(X, out["grad"]),
        "cons": lambda: M.eval_cons(X, out["c"]),
        "jac": lambda: M.eval_jac(X, out["jvals"]),
        "hess": lambda: M.eval_hess(X, LAM, pt.sigma, out["hvals"]),
        "jtprod": lambda: M.jtprod(X, LAM, out["jtv"]),
        "condensed": lambda: M.assemble_condensed(out["hvals"], out["jvals"], DX, D, out["kvals"]),
        "jhk": lambda: M.eval_jhk(X, LAM, pt.sigma, DX, D, out["jvals"], out["hvals"], out["kvals"]),
    }
    # lifted-KKT calls around K (Sec. III-B) on one interior iterate inside
    # the model's bounds
    bnd = [torch.empty(k, dtype=torch.float64, device=dev) for k in (M.n, M.n, M.m, M.m)]
    M.bounds(*bnd)
    sh = synth.make_ipm_state(*(b.cpu().numpy() for b in bnd), seed=3)
    del bnd
    tt = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    keep = {f: tt(getattr(sh, f)) for f in ("x", "s", "y", "zl", "zu", "vl", "vu", "xl", "xu", "sl", "su")}
    st = M.ipm_state(**keep, mu=sh.mu, delta_w=sh.delta_w, delta_c=sh.delta_c)
    del sh
    e = lambda k: torch.empty(k, dtype=torch.float64, device=dev)
    rhs, jvo, dxo, dco = e(M.n), e(M.m), e(M.n), e(M.m)
    rec = [e(M.m), e(M.m), e(M.n), e(M.n), e(M.m), e(M.m)]
    calls["jprod"] = lambda: M.jprod(keep["x"], X, jvo)
    calls["condensed_rhs"] = lambda: M.condensed_rhs(st, out["grad"], out["c"], dxo, dco, rhs)
    calls["recover_step"] = lambda: M.recover_step(st, out["c"], rhs, *rec)
    per = {}
    for name, fn in calls.items():
        t = event_time(torch, fn, args.call_reps)
        per[name] = {"ms": round(t, 4), "gbs": round(by[name] / t / 1e6, 1)}
    graph_ms = event_time(torch, lambda: M.sweep_graph(sa), args.call_reps)
    jhk_ms = per["jhk"]["ms"]
    sweep_bytes = kb["sweep"]
    res = {
        "value": nnz / (ms / 1e3),
        "ms_per_step": ms,
        "config": {"workload": "paper-scale multi-period AC OPF evaluation sweep (synthetic grid)",
                   "N": net.N, "B": net.B, "G": net.G, "T": net.T, "n": M.n, "m": M.m,
                   "nnz_jac": M.nnz_jac, "nnz_hess": M.nnz_hess, "nnz_kkt": M.nnz_kkt, "seed": 3},
        "hbm_gbs": sweep_bytes / (ms / 1e3) / 1e9,
        "sweep_bytes": sweep_bytes,
        "graph_sweep_ms": round(graph_ms, 4),
        "median_step_ms": round(median_step_ms, 4),
        "eager_sweep_ms": round(eager_ms, 4),
        # Jacobian + Hessian + condensed matrix alone (opf_eval_jhk): nnz/s,
        # its rate in its own algorithmic bytes (what the fused pass must
        # move), and the effective rate in the separate pipeline's bytes (J
        # and H written, then read back by the condensation: 3.56 GB, which
        # the fused pass never moves)
        "jhk": {"ms": jhk_ms, "nnz_per_s": nnz / (jhk_ms / 1e3),
                "own_bytes": by["jhk"], "own_frac_of_peak": round(by["jhk"] / jhk_ms / 1e6 / HBM_PEAK_GBS, 4),
                "separate_pipeline_bytes": by["jac"] + by["hess"] + by["condensed"],
                "separate_pipeline_effective_frac": round((by["jac"] + by["hess"] + by["condensed"]) / jhk_ms
                                                          / 1e6 / HBM_PEAK_GBS, 4)},
        "calls": per,
        "separate_jhk_ms": round(per["jac"]["ms"] + per["hess"]["ms"] + per["condensed"]["ms"], 4),
        "kernels": kernels,
        "symbolic": symbolic,
    }
    cp = args.copy_peak
    kt = kernels["sweep_a"]["median_ms"]
    ach = kb["sweep_a"] / kt / 1e6
    res["roofline"] = {"bound": "hbm", "kernel": "k_sweep_a (lines and generators of the fused sweep)",
                       "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4),
                       "measured_copy_gbs": cp["gbs"], "frac_of_measured_copy": round(ach / cp["gbs"], 4),
                       "algorithmic_bytes": kb["sweep_a"], "median_ms": kt, "traffic": profiled_traffic("k_sweep_a"),
                       "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"}
    kt_b = kernels["sweep_b"]["median_ms"]
    res["roofline_bus"] = {"kernel": "k_sweep_b", "achieved": round(kb["sweep_b"] / kt_b / 1e6, 1),
                           "frac": round(kb["sweep_b"] / kt_b / 1e6 / HBM_PEAK_GBS, 4),
                           "algorithmic_bytes": kb["sweep_b"], "median_ms": kt_b,
                           "traffic": profiled_traffic("k_sweep_b")}
    sweep_gbs = sweep_bytes / (median_step_ms / 1e3) / 1e9
    res["sweep_roofline"] = {"algorithmic_bytes": sweep_bytes, "median_step_ms": round(median_step_ms, 4),
                             "achieved": round(sweep_gbs, 1), "frac": round(sweep_gbs / HBM_PEAK_GBS, 4),
                             "frac_of_measured_copy": round(sweep_gbs / cp["gbs"], 4),
                             "jhk_separate_pipeline_effective_frac": round(
                                 (by["jac"] + by["hess"] + by["condensed"]) / median_step_ms / 1e6 / HBM_PEAK_GBS, 4)}
    M.close()
    return res


FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 (vector and matrix cores alike)


def bench_chol(torch, dev, args):
    """Static-pivot sparse Cholesky of the paper-scale condensed matrix (the
    linear solve of one interior-point iteration, Sec. III-B): analysis
    once, then factor and solve timed with events on the model's stream.
    K from the evaluation path at an iterate with an objective-only
    Hessian and diag_x, D ~ logU(1e-4, 1e4), so K is positive definite."""
    from paper_2405_14032_amd import capi, synth
    net = synth.config_network("paper")
    pt = synth.make_point(net, 3)
    M = capi.Model([net], device=0)
    M.use_current_torch_stream()
    rng = np.random.default_rng(17)
    tt = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    X = tt(pt.x)
    LAM = torch.zeros(M.m, dtype=torch.float64, device=dev)
    DX, D = tt(10.0 ** rng.uniform(-4, 4, M.n)), tt(10.0 ** rng.uniform(-4, 4, M.m))
    e = lambda k: torch.empty(k, dtype=torch.float64, device=dev)
    jv, hv, kv = e(M.nnz_jac), e(M.nnz_hess), e(M.nnz_kkt)
    M.eval_jhk(X, LAM, 1.0, DX, D, jv, hv, kv)
    del jv, hv, DX, D
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = capi.Chol(M)
    analyze_s = time.perf_counter() - t0
    info = F.info()
    npert = torch.zeros(1, dtype=torch.int32, device=dev)
    B, XS = tt(rng.standard_normal(M.n)), e(M.n)
    fac_ms = event_time(torch, lambda: F.factor(kv, 0.0, 1.0, npert), 2)
    sol_ms = event_time(torch, lambda: F.solve(B, XS), 3)
    perturbed = int(npert.item())
    tflops = info["flops"] / (fac_ms / 1e3) / 1e12
    res = {"workload": "paper-scale condensed matrix K (n = %d, nnz(lower K) = %d)" % (M.n, M.nnz_kkt),
           "analysis_s": round(analyze_s, 3), "factor_ms": round(fac_ms, 2), "solve_ms": round(sol_ms, 2),
           "factor_tflops": round(tflops, 2), "flops": info["flops"], "flops_interior": info["flops_interior"],
           "factor_entries": info["factor_entries"], "fronts_per_period": info["nodes"],
           "large_fronts": info["large_nodes"], "periods_per_chunk": info["chunk"],
           "static_pivots": perturbed,
           "roofline": {"bound": "fp64", "achieved": round(tflops, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
                        "note": "whole factorization: algorithmic flops / factor time"}}
    F.close()
    M.close()
    return res


def bench_ipm(torch, dev, args):
    """The lifted-KKT interior-point loop (opf_ipm_solve, filter line
    search): a whole solve to 1e-4 of the 2000-bus, 24-period grid with its
    loads capped at 30 % of the generation capacity (synth.cap_load), timed
    after one warm-up solve; the same grid with its loads as drawn (the
    loop's status: converged or stalled); the capped grid over 168 periods
    (one solve); and the cost of one iteration at paper scale (three
    iterations timed; evaluation + condensation, factorization, solve +
    recovery)."""
    from paper_2405_14032_amd import capi, synth
    out = {}
    net = synth.config_network("mid")
    M = capi.Model([net], device=0)
    M.use_current_torch_stream()
    F = capi.Chol(M)
    x = torch.empty(M.n, dtype=torch.float64, device=dev)
    r = capi.ipm_solve(M, F, x, max_iter=150)
    out["whole_solve_uncapped"] = {"workload": "N=2000 B=3200 G=400 T=24 (seed 2), loads as drawn, tol 1e-4",
                                   "n": M.n, "m": M.m, "status": r["status_name"], "iterations": r["iterations"],
                                   "seconds": round(r["seconds"], 3), "theta": r["theta"], "err": r["err"],
                                   "objective": r["objective"]}
    log(f"ipm uncapped mid solve: {out['whole_solve_uncapped']}")
    F.close()
    M.close()
    net = synth.cap_load(synth.config_network("mid"), 0.3)
    M = capi.Model([net], device=0)
    M.use_current_torch_stream()
    F = capi.Chol(M)
    x = torch.empty(M.n, dtype=torch.float64, device=dev)
    capi.ipm_solve(M, F, x)
    r = capi.ipm_solve(M, F, x)
    out["whole_solve"] = {"workload": "N=2000 B=3200 G=400 T=24 (seed 2), loads capped at 0.3 of capacity, tol 1e-4",
                          "n": M.n, "m": M.m, "converged": bool(r["converged"]), "status": r["status_name"],
                          "iterations": r["iterations"], "factorizations": r["factorizations"],
                          "seconds": round(r["seconds"], 4), "s_per_iteration": round(r["seconds"] / max(1, r["iterations"]), 4),
                          "objective": r["objective"]}
    F.close()
    M.close()
    # the same grid over a week of hourly periods (n = 2956800), one solve
    net = synth.cap_load(synth.make_network(2000, 3200, 400, 168, 2), 0.3)
    M = capi.Model([net], device=0)
    M.use_current_torch_stream()
    F = capi.Chol(M)
    x = torch.empty(M.n, dtype=torch.float64, device=dev)
    r = capi.ipm_solve(M, F, x)
    out["whole_solve_week"] = {"workload": "N=2000 B=3200 G=400 T=168 (seed 2), loads capped at 0.3 of capacity, tol 1e-4",
                               "n": M.n, "m": M.m, "converged": bool(r["converged"]), "status": r["status_name"],
                               "iterations": r["iterations"], "factorizations": r["factorizations"],
                               "seconds": round(r["seconds"], 3), "factor_s": round(r["t_factor"], 3),
                               "solve_recover_s": round(r["t_solve"], 3), "objective": r["objective"]}
    log(f"ipm week solve: {out['whole_solve_week']}")
    F.close()
    M.close()
    net = synth.config_network("paper")
    M = capi.Model([net], device=0)
    M.use_current_torch_stream()
    F = capi.Chol(M)
    x = torch.empty(M.n, dtype=torch.float64, device=dev)
    r = capi.ipm_solve(M, F, x, max_iter=3)
    k = max(1, r["iterations"])
    out["paper_iteration"] = {"workload": "paper-scale grid, first 3 iterations", "n": M.n, "m": M.m,
                              "s_per_iteration": round(r["seconds"] / k, 3),
                              "eval_condense_s": round(r["t_eval"] / k, 4), "factor_s": round(r["t_factor"] / k, 3),
                              "solve_recover_s": round(r["t_solve"] / k, 3)}
    F.close()
    M.close()
    return out


def bench_paper_solve(torch, dev, cap):
    """A whole interior-point solve (tol 1e-4) of the paper-scale grid with
    every period's loads scaled so that the peak period draws ``cap`` of the
    generation capacity (synth.cap_load); one progress line per iteration on
    stderr."""
    from paper_2405_14032_amd import capi, synth
    net = synth.cap_load(synth.config_network("paper"), cap)
    t0 = time.perf_counter()
    M = capi.Model([net], device=0)
    M.use_current_torch_stream()
    F = capi.Chol(M)
    setup_s = time.perf_counter() - t0
    x = torch.empty(M.n, dtype=torch.float64, device=dev)
    r = capi.ipm_solve(M, F, x, max_iter=200, verbose=1)
    out = {"workload": f"paper-scale grid N=10000 B=13000 G=2000 T=168 (seed 3), loads capped at {cap} of capacity, "
                       "tol 1e-4", "n": M.n, "m": M.m, "setup_s": round(setup_s, 2), "converged": bool(r["converged"]),
           "status": r["status_name"], "iterations": r["iterations"], "factorizations": r["factorizations"],
           "seconds": round(r["seconds"], 2),
           "eval_s": round(r["t_eval"], 2),
           "factor_s": round(r["t_factor"], 2), "solve_recover_s": round(r["t_solve"], 2),
           "objective": r["objective"], "err": r["err"]}
    F.close()
    M.close()
    return out


def bench_batched(torch, dev, args):
    from paper_2405_14032_amd import capi, synth
    nets = synth.batched_networks(64)
    pts = [synth.make_point(n, synth.BATCH_SEED0 + k) for k, n in enumerate(nets)]
    log(f"batched: 64 instances, sum n = {sum(n.n for n in nets)}")
    MB = capi.Model(nets, device=0)
    MB.use_current_torch_stream()
    MB.autotune(args.tune_cache)
    cat = lambda key: np.concatenate([getattr(p, key) for p in pts])
    pb = type("P", (), {})()
    pb.x, pb.lam, pb.diag_x, pb.dcon = cat("x"), cat("lam"), cat("diag_x"), cat("dcon")
    X, LAM, DX, D = make_inputs(torch, dev, None, pb)
    ob = outputs(torch, dev, MB)
    sb = MB.sweep_args(x=X, lam=LAM, sigma=1.0, v=LAM, diag_x=DX, dcon=D, **ob)
    plain = []
    for k, (net, pt) in enumerate(zip(nets, pts)):
        Mk = capi.Model([net], device=0)
        Mk.use_current_torch_stream()
        xs = make_inputs(torch, dev, net, pt)
        ok = outputs(torch, dev, Mk)
        plain.append((Mk, xs, ok, Mk.sweep_args(x=xs[0], lam=xs[1], sigma=1.0, v=xs[1], diag_x=xs[2],
                                                 dcon=xs[3], **ok)))

    def run_plain():
        for Mk, _, _, sk in plain:
            Mk.sweep(sk)

    g_ms = event_time(torch, lambda: MB.sweep_graph(sb), args.call_reps)
    e_ms = event_time(torch, lambda: MB.sweep(sb), args.call_reps)
    p_ms = event_time(torch, run_plain, max(2, args.call_reps // 4))
    torch.cuda.synchronize()
    # agreement: element values bit-identical, objective within 1e-12
    worst_f = 0.0
    identical = True
    for k, (Mk, _, ok, _) in enumerate(plain):
        for key, offs in (("grad", MB.x_off), ("c", MB.c_off), ("jvals", MB.j_off), ("hvals", MB.h_off),
                          ("jtv", MB.x_off), ("kvals", MB.k_off)):
            a = ob[key][offs[k]:offs[k + 1]]
            identical &= bool(torch.equal(a, ok[key]))
        fb, fp = float(ob["f"][k]), float(ok["f"][0])
        worst_f = max(worst_f, abs(fb - fp) / max(abs(fp), 1e-300))
    nnz = MB.nnz_jac + MB.nnz_hess + MB.nnz_kkt
    # the batched sweep's own algorithmic bytes: the sum of its instances'
    sweep_bytes = sum(sweep_kernel_bytes(net, Mk, 0)["sweep"] for net, (Mk, *_) in zip(nets, plain))
    gbs = sweep_bytes / (g_ms / 1e3) / 1e9
    res = {"instances": 64, "sum_n": MB.n, "graph_ms": round(g_ms, 4), "eager_ms": round(e_ms, 4),
           "plain_64_ms": round(p_ms, 4), "speedup_vs_plain": round(p_ms / g_ms, 3),
           "nnz_per_s": nnz / (g_ms / 1e3), "sweep_bytes": sweep_bytes, "hbm_gbs": round(gbs, 1),
           "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
           "launches": "one HIP graph of two tile-list kernels (line/generator pass with the objective's "
                       "partials, bus pass with its sums) over all 64 instances, one block per tile",
           "elements_bit_identical": identical, "objective_max_rel_diff": worst_f}
    for Mk, *_ in plain:
        Mk.close()
    MB.close()
    return res


def bench_adjoint(torch, dev, args):
    from paper_2405_14032_amd import capi, synth
    from paper_2405_14032_amd.autograd import OpfCons
    nets = synth.adjoint_networks(16)
    pts = [synth.make_point(n, synth.ADJOINT_SEED0 + k) for k, n in enumerate(nets)]
    log("adjoint: 16 mid instances")
    MA = capi.Model(nets, device=0)
    MA.use_current_torch_stream()
    MA.autotune(args.tune_cache)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    X = t(np.concatenate([p.x for p in pts])).requires_grad_(True)
    PD = t(np.concatenate([n.pd.reshape(-1) for n in nets])).requires_grad_(True)
    QD = t(np.concatenate([n.qd.reshape(-1) for n in nets])).requires_grad_(True)
    LAM = t(np.concatenate([p.lam for p in pts]))

    def fused():
        X.grad = PD.grad = QD.grad = None
        c = OpfCons.apply(X, PD, QD, MA)
        c.backward(LAM)

    # plain per-instance path: eval_cons, eval_jac + COO product, load slice
    plain = []
    for k, (net, pt) in enumerate(zip(nets, pts)):
        Mk = capi.Model([net], device=0)
        Mk.use_current_torch_stream()
        rows = torch.empty(Mk.nnz_jac, dtype=torch.int32, device=dev)
        cols = torch.empty(Mk.nnz_jac, dtype=torch.int32, device=dev)
        Mk.jac_structure(rows, cols)
        a, b = MA.c_off[k], MA.c_off[k + 1]
        xk = X.detach()[MA.x_off[k]:MA.x_off[k + 1]]
        lk = LAM[a:b]
        pdk = PD.detach()[k * net.T * net.N:(k + 1) * net.T * net.N]
        qdk = QD.detach()[k * net.T * net.N:(k + 1) * net.T * net.N]
        plain.append(dict(M=Mk, rows=rows.long(), cols=cols.long(), x=xk, lam=lk, pd=pdk, qd=qdk,
                          jv=torch.empty(Mk.nnz_jac, dtype=torch.float64, device=dev),
                          c=torch.empty(Mk.m, dtype=torch.float64, device=dev),
                          g=torch.zeros(Mk.n, dtype=torch.float64, device=dev), net=net))

    def run_plain():
        for p in plain:
            M, net = p["M"], p["net"]
            M.set_load(p["pd"], p["qd"])
            M.eval_cons(p["x"], p["c"])
            M.eval_jac(p["x"], p["jv"])
            p["g"].zero_()
            p["g"].index_add_(0, p["cols"], p["jv"] * p["lam"][p["rows"]])
            mp = 2 * net.N + 7 * net.B + 1
            lam_t = p["lam"][:net.T * mp].view(net.T, mp)
            p["gpd"] = -lam_t[:, :net.N]
            p["gqd"] = -lam_t[:, net.N:2 * net.N]

    f_ms = event_time(torch, fused, args.call_reps)
    p_ms = event_time(torch, run_plain, max(2, args.call_reps // 4))
    torch.cuda.synchronize()
    worst = 0.0
    for k, p in enumerate(plain):
        a = X.grad[MA.x_off[k]:MA.x_off[k + 1]]
        worst = max(worst, float(((a - p["g"]).abs() / (1 + p["g"].abs())).max()))
    res = {"instances": 16, "fused_fwd_bwd_ms": round(f_ms, 4), "plain_ms": round(p_ms, 4),
           "speedup_vs_plain": round(p_ms / f_ms, 3), "jtv_max_rel_diff_vs_plain": worst}
    for p in plain:
        p["M"].close()
    MA.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--call-reps", type=int, default=20)
    ap.add_argument("--tune-cache", default=TUNE_CACHE)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-plain", action="store_true", help="skip the batched and adjoint legs")
    ap.add_argument("--no-chol", action="store_true", help="skip the sparse Cholesky leg")
    ap.add_argument("--chol-only", action="store_true",
                    help="run only the sparse Cholesky leg and print its JSON object (for profiling)")
    ap.add_argument("--paper-solve", type=float, default=None, metavar="CAP",
                    help="run only a whole interior-point solve of the paper-scale grid with its loads capped at "
                         "CAP of the generation capacity (several minutes) and print its JSON object")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="accepted for older profiling commands; the 1 GiB copy now always runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the evaluation path has no "
              "multi-GPU mode", file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not (args.no_cpu_baseline or args.chol_only or args.paper_solve is not None):
        # before anything initialises the GPU: the oracle's workers are fresh
        # interpreters started from this process
        log("cpu baseline (oracle on the host cores) ...")
        cpu = cpu_baseline()
        log(f"cpu baseline: {cpu['value']:.3e} nnz/s on {cpu['cores']} cores ({cpu['cpu_model']})")
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    os.makedirs(os.path.dirname(args.tune_cache), exist_ok=True)
    # the plain 1 GiB copy: the measured HBM peak, and the reference kernel
    # of the counter calibration (its FETCH_SIZE / WRITE_SIZE per dispatch)
    args.copy_peak = copy_peak(torch, dev)
    log(f"1 GiB device copy: {args.copy_peak}")
    if args.chol_only:
        print(json.dumps({"chol": bench_chol(torch, dev, args)}), flush=True)
        return
    if args.paper_solve is not None:
        print(json.dumps({"paper_solve": bench_paper_solve(torch, dev, args.paper_solve)}), flush=True)
        return
    res = bench_plain(torch, dev, args)
    log(f"plain sweep: {res['ms_per_step']:.3f} ms/step")
    line = {"metric": METRIC, "value": res["value"], "unit": "nnz/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic (seeded grids standing in for the paper's public cases)",
            "config": res["config"], "hbm_gbs": res["hbm_gbs"], "sweep_bytes": res["sweep_bytes"],
            "graph_sweep_ms": res["graph_sweep_ms"], "median_step_ms": res["median_step_ms"],
            "eager_sweep_ms": res["eager_sweep_ms"], "hbm_copy": args.copy_peak,
            "sweep_roofline": res["sweep_roofline"],
            "jhk": res["jhk"], "separate_jhk_ms": res["separate_jhk_ms"],
            "calls": res["calls"], "kernels": res["kernels"], "symbolic": res["symbolic"], "roofline": res["roofline"],
            "roofline_bus": res["roofline_bus"]}
    if not args.no_chol:
        line["chol"] = bench_chol(torch, dev, args)
        log(f"chol: {line['chol']}")
        line["ipm"] = bench_ipm(torch, dev, args)
        log(f"ipm: {line['ipm']}")
    if not args.only_plain:
        line["batched"] = bench_batched(torch, dev, args)
        log(f"batched: {line['batched']}")
        line["adjoint"] = bench_adjoint(torch, dev, args)
        log(f"adjoint: {line['adjoint']}")
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
