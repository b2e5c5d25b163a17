"""Benchmark: level-blocked MPK vs p back-to-back SpMVs on one MI355X.

Workload: 27-point stencil on a 160^3 grid (N = 4,096,000, nnz = 109,215,352),
off-diagonal values U[-1, 1], dominant diagonal, rows randomly relabelled,
x ~ U[-1, 1]; powers p = 8 (headline) with p = 4 and 6 reported alongside.
Inputs are generated on the host from a seed and are resident in HBM before
the timed region starts.

One step = one call of the hot path: mpk_run computing y_1..y_p.  Reported:
MPK GFLOP/s (2 nnz p / t), speedup over the faster of two tuned baselines
(p SpMV launches on the matrix as given, and on the BFS-renumbered matrix),
roofline fraction of the persistent kernel against 8 TB/s HBM on algorithmic
bytes, mixed-precision (FP32 / BF16 values, FP32 or FP64 arithmetic)
throughput and error against the FP64 run, the synchronisation ladder,
refined plans (recursion, s_m = 1, 2) and bulky-level matrices, and the FP64
CPU oracle timed on the host (the only use of the oracle here).  Every MPK
configuration reported is the autotuner's pick among a few candidates.
Other workloads: 64^2 Laplacian, Anderson 128^3 and heat-equation 160^3
Chebyshev propagation, multi-RHS RGG, a thin-level 2D 9-point 4096^2
stencil, the learned tuner.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MPK GFLOP/s & speedup vs p× SpMV (same GPU), FP64 and mixed precision"
HBM_PEAK_GBS = 8000.0


PROFILE = os.path.join(ROOT, "profiles", "mpk_persistent_27pt160_p8.txt")


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("kernels.h", "mpk_device.hip"):
        with open(os.path.join(ROOT, "paper_2205_01598_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(key: str = "traffic_bytes_per_launch"):
    """HBM-side bytes per launch from the committed counter summary (the MPK
    kernel's, or with key spmv_traffic_bytes_per_launch one baseline SpMV's),
    if it was taken on the kernel sources as they are now (else None)."""
    try:
        kv = {}
        with open(PROFILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_hash") != kernel_source_hash():
            return None
        return int(kv[key])
    except (OSError, KeyError, ValueError):
        return None


def code_balance(n, nnz, p):
    """Code balance B_C (Sec. 3): bytes moved per flop, 2 nnz flops per SpMV.
    Algorithmic (matrix once, x, p outputs) and measured from the profiled
    L2-to-fabric traffic, for the MPK and for p baseline SpMVs; None where no
    profile of the current sources exists."""
    flops = 2.0 * nnz * p
    t_mpk, t_spmv = profiled_traffic(), profiled_traffic("spmv_traffic_bytes_per_launch")
    return {"algorithmic_mpk": round(mpk_bytes(n, nnz, p) / flops, 4),
            "algorithmic_p_spmvs": round(p * spmv_bytes(n, nnz) / flops, 4),
            "measured_mpk": None if t_mpk is None else round(t_mpk / flops, 4),
            "measured_p_spmvs": None if t_spmv is None else round(p * t_spmv / flops, 4),
            "unit": "bytes/flop"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def mpk_bytes(n, nnz, p, k=1, vbytes=8):
    # matrix once (values + int32 columns + int32 row pointers), y_0 read,
    # y_1..y_p written
    return (vbytes + 4) * nnz + 4 * (n + 1) + 8 * n * k + 8 * p * n * k


def spmv_bytes(n, nnz, k=1, vbytes=8):
    return (vbytes + 4) * nnz + 4 * (n + 1) + 16 * n * k


def timed_each(torch, fn, min_seconds=1.0, max_runs=2000, before=None):
    """Times single calls with events until at least `min_seconds` of GPU
    time has been measured; `before` (untimed) runs ahead of every call.
    Returns (mean, min, median) in ms and the number of calls."""
    ts = []
    while sum(ts) < min_seconds * 1e3 and len(ts) < max_runs:
        if before is not None:
            before()
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        e.synchronize()
        ts.append(s.elapsed_time(e))
    return float(np.mean(ts)), float(np.min(ts)), float(np.median(ts)), len(ts)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_errs(Y, ref):
    return [float(np.linalg.norm(Y[q] - ref[q]) / np.linalg.norm(ref[q])) for q in range(ref.shape[0])]


def oracle_threads():
    """Host threads for the oracle's row-parallel variant: every core this
    process may run on, capped by OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(cap))) if cap.isdigit() and int(cap) > 0 else n


def fmt(v):
    return float(f"{v:.3e}")


def bench_small_2d(torch, Plan, W, dev):
    """64 x 64 5-point Laplacian, p = 4 (cache- and launch-latency-bound).
    The synchronisation ladder runs on many small level groups (C = 64 KB,
    49 groups), where it shows what point-to-point flags save over kernel
    boundaries; the MPK itself is timed in the fastest of a few (C, skew,
    tile, grid) settings, like every other leg, and checked in that setting
    against the oracle and bit for bit against the baseline."""
    import oracle as O

    A = W.stencil_2d(64, 5)
    x = W.uniform_vector(A.n, seed=0)
    pl = Plan(A, 4, 64 * 1024, root_mode=1, tile_nnz=2048)
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    Y = torch.empty((4, A.n), dtype=torch.float64, device=dev)
    tb = timed(torch, lambda: pl.run_baseline(X, Y), 200, 20)
    Yb = Y.clone()
    t_ladder = timed(torch, lambda: pl.run(X, Y), 200, 20)
    pl.status()
    G = pl.info()["n_groups"]
    ladder = {"level_groups": G,
              "launch_per_node_us": round(timed(torch, lambda: pl.run_sync(X, Y, "node"), 100, 10) * 1e3, 2),
              "launch_per_wavefront_us": round(timed(torch, lambda: pl.run_sync(X, Y, "wavefront"), 100, 10) * 1e3, 2),
              "p2p_flags_us": round(t_ladder * 1e3, 2)}
    cands = [(64 * 1024, 1, 2048, 0), (1 << 20, 2, 1024, 64), (1 << 20, 4, 1024, 64), (64 << 20, 1, 1024, 64),
             (64 << 20, 2, 2048, 64)]
    runs = {}
    for cb, skew, tile, wg in cands:
        pl.retune(4, cb, root_mode=1, skew=skew, tile_nnz=tile, workgroups=wg)
        runs[(cb, skew, tile, wg)] = timed(torch, lambda: pl.run(X, Y), 200, 20)
        pl.status()
    best = min(runs, key=runs.get)
    cb, skew, tile, wg = best
    pl.retune(4, cb, root_mode=1, skew=skew, tile_nnz=tile, workgroups=wg)
    tm = timed(torch, lambda: pl.run(X, Y), 200, 20)
    pl.status()
    Yo = np.empty((4, A.n))
    Yo[:, perm] = Y.cpu().numpy()
    parity = {"max_rel_err_vs_oracle": fmt(max(rel_errs(Yo, O.spmv_powers(A, x, 4)))),
              "bit_equal_to_baseline": bool(torch.equal(Y, Yb))}
    return {"workload": "5-point Laplacian 64^2, p=4", "mpk_us": round(tm * 1e3, 2),
            "baseline_us": round(tb * 1e3, 2), "speedup": round(tb / tm, 3),
            "config": {"cache_bytes": cb, "skew": skew, "tile_nnz": tile, "workgroups": wg,
                       "level_groups": pl.info()["n_groups"]},
            "runs_us": {f"C{k[0]}_s{k[1]}_t{k[2]}_wg{k[3]}": round(v * 1e3, 2) for k, v in runs.items()},
            "sync_ladder": ladder, "parity": parity}


def plan_device_only(args):
    """Plans the headline matrix from its CSR in device memory twice (the
    second one timed), for a kernel trace of the device planner."""
    import torch

    import workloads as W
    from paper_2205_01598_amd import Plan

    A, _ = W.stencil_27pt_random(args.n, seed=args.seed)
    dA = [torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in (A.rowptr, A.col, A.val)]
    secs = []
    pl = None
    for _ in range(2):
        del pl  # the previous plan is freed before the clock starts
        torch.cuda.synchronize()
        t0 = time.time()
        pl = Plan.from_device(*dA, args.p, 256 << 20, root_mode=1)
        torch.cuda.synchronize()
        secs.append(time.time() - t0)
    inf = pl.info()
    del pl
    # a third plan with the upload (schedule tables to the device) timed apart
    torch.cuda.synchronize()
    t0 = time.time()
    pl3 = Plan.from_device(*dA, args.p, 256 << 20, root_mode=1, upload=False)
    t1 = time.time()
    pl3.upload()
    torch.cuda.synchronize()
    t2 = time.time()
    print(json.dumps({"plan_seconds": [round(v, 4) for v in secs], "levels": inf["n_levels"],
                      "phase_seconds": [round(v, 4) for v in inf["phase_seconds"]],
                      "create_seconds": round(t1 - t0, 4), "upload_seconds": round(t2 - t1, 4)}), flush=True)


def only_config(args):
    """The headline matrix in one plan configuration, `steps` timed runs after
    `warmup` (rocprofv3 runs of a single configuration)."""
    import torch

    import workloads as W
    from paper_2205_01598_amd import Plan

    sm, cmb, skew, tile, streams = (int(v) for v in args.only_config.split(","))
    A, _ = W.stencil_27pt_random(args.n, seed=args.seed)
    x = W.uniform_vector(A.n, seed=args.seed)
    pl = Plan(A, args.p, cmb << 20, root_mode=1, skew=skew, tile_nnz=tile, xcd_streams=streams,
              recursion_stages=sm)
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).cuda()
    Y = torch.empty((args.p, A.n), dtype=torch.float64, device="cuda")
    ms = timed(torch, lambda: pl.run(X, Y), args.steps, args.warmup)
    pl.status()
    inf = pl.info()
    print(json.dumps({"config": args.only_config, "ms": round(ms, 4), "units": inf["n_units"],
                      "tiles": inf["n_tiles"]}), flush=True)


def bench_chebyshev(torch, Plan, W, dev, steps_err=10):
    """Anderson 128^3, degree-32 Chebyshev step as 4 MPK blocks of p = 8.
    Every configuration the autotuner picks is checked in the same run: one
    step of the MPK equals the baseline's bit for bit, and ten steps are
    compared with ten steps of the FP64 oracle (relative error per step)."""
    import oracle as O
    from paper_2205_01598_amd import tune
    from paper_2205_01598_amd.cheb import ChebPropagator

    A = W.anderson_3d(128, seed=0)
    x = W.random_phase_state(A.n, seed=0)
    M, p, r_dt = 32, 8, 10.0
    out = {"workload": "Anderson 128^3 (W=16, open BC, A=H/14), degree 32, p=8, r*dt=10, complex state"}
    t0 = time.time()
    coeffs = O.cheb_coefficients(M, r_dt)
    ref, state = [], x
    for _ in range(steps_err):
        state = O.cheb_propagate(A, state, coeffs, threads=oracle_threads())
        ref.append(state)
    log(f"chebyshev oracle: {steps_err} steps in {time.time() - t0:.1f}s")
    for dt in ("f64", "f32", "bf16"):
        pl = Plan(A, p, 256 << 20, root_mode=1, nrhs=2, val_dtype=dt, skew=2, tile_nnz=8192)
        perm = pl.arrays()[0].astype(np.int64)
        prop = ChebPropagator.schroedinger(pl, M, r_dt)
        X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
        acc = torch.empty_like(X)
        tb = timed(torch, lambda: prop.step(X, acc, baseline=True), 20, 3)
        acc_base = acc.clone()
        # the autotuner over a few (C, tile, skew); the matrix fits the
        # Infinity Cache, so smaller budgets than the headline's are tried
        cands = [dict(cache_mb=C, tile_nnz=t, skew=s) for C, t, s in
                 ((256, 8192, 2), (128, 4096, 2), (64, 2048, 2), (32, 4096, 12), (64, 8192, 12))]
        cfg = tune.autotune(torch, pl, p, cands, lambda: prop.step(X, acc), reps=10, nrhs=2, val_dtype=dt)[0]
        tm = timed(torch, lambda: prop.step(X, acc), 20, 3)
        pl.status()
        ent = {"step_ms": round(tm, 4), "baseline_step_ms": round(tb, 4), "speedup": round(tb / tm, 3),
               "gflops": round(2.0 * A.nnz * 2 * M / tm / 1e6, 1),
               "config": cfg, "bit_equal_to_baseline": bool(torch.equal(acc, acc_base))}
        if dt == "f64":
            # the fixed cost of the persistent kernel: one level group (no
            # reuse window), then back to the pick
            pl.retune(p, 64 << 30, root_mode=1, nrhs=2, val_dtype=dt, skew=2, tile_nnz=8192)
            ent["one_level_group"] = {"groups": pl.info()["n_groups"],
                                      "step_ms": round(timed(torch, lambda: prop.step(X, acc), 20, 3), 4)}
            pl.status()
            tune.autotune(torch, pl, p, [cfg], lambda: prop.step(X, acc), reps=1, warmup=0, nrhs=2, val_dtype=dt)
            # the working set fits the 256 MB Infinity Cache: also time each
            # step after reading 512 MB of other data
            scrub = torch.ones(64 << 20, dtype=torch.float64, device=dev)
            sink = torch.empty((), dtype=torch.float64, device=dev)
            wipe = lambda: sink.copy_(scrub.sum())  # noqa: E731
            sm = timed_each(torch, lambda: prop.step(X, acc), 0.1, 40, before=wipe)[0]
            sb = timed_each(torch, lambda: prop.step(X, acc, baseline=True), 0.1, 40, before=wipe)[0]
            ent["cache_scrubbed"] = {"step_ms": round(sm, 4), "baseline_step_ms": round(sb, 4),
                                     "speedup": round(sb / sm, 3)}
            del scrub, sink
        states, state = [], X
        for _ in range(steps_err):
            nxt = torch.empty_like(state)
            prop.step(state, nxt)
            h = np.empty((A.n, 2))
            h[perm] = nxt.cpu().numpy()
            states.append(h)
            state = nxt
        ent["rel_err_vs_oracle_per_step"] = [fmt(np.linalg.norm(a - b) / np.linalg.norm(b))
                                             for a, b in zip(states, ref)]
        ent["norm_after_steps"] = float(f"{np.linalg.norm(states[-1]):.12f}")
        out[dt] = ent
        del pl, prop
    return out


def bench_heat(torch, Plan, W, dev):
    """Heat equation on 160^3 with finite differences of order 2, 4, 6
    (Table 3), degree-32 Chebyshev step (tau = 70, coefficients below 1e-4
    from degree 32 on) as 4 MPK blocks of p = 8, real coefficients."""
    import oracle as O
    from paper_2205_01598_amd.cheb import ChebPropagator, degree_for_cutoff

    M, p, tau = 32, 8, 70.0
    assert degree_for_cutoff(tau, kind="heat") <= M
    out = {"workload": "heat equation 160^3, order 2/4/6 finite differences, A = L/r - I, degree 32, p=8, tau=70"}
    x = W.uniform_vector(160 ** 3, seed=0)
    for order in (2, 4, 6):
        A, r = W.heat_operator_3d(160, order)
        pl = Plan(A, p, 256 << 20, root_mode=1, skew=2, tile_nnz=8192)
        perm = pl.arrays()[0].astype(np.int64)
        prop = ChebPropagator.heat(pl, M, tau)
        X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
        acc = torch.empty_like(X)
        accb = torch.empty_like(X)
        tm = timed(torch, lambda: prop.step(X, acc), 10, 2)
        tb = timed(torch, lambda: prop.step(X, accb, baseline=True), 10, 2)
        pl.status()
        diff = float((acc - accb).norm() / accb.norm())
        ref = O.cheb_propagate_real(A, x, O.heat_coefficients(M, tau), threads=oracle_threads())
        h = np.empty(A.n)
        h[perm] = acc.cpu().numpy()
        out[f"order{order}"] = {"nnz": A.nnz, "step_ms": round(tm, 4), "baseline_step_ms": round(tb, 4),
                                "speedup": round(tb / tm, 3), "gflops": round(2.0 * A.nnz * M / tm / 1e6, 1),
                                "mpk_vs_baseline_rel_diff": float(f"{diff:.3e}"),
                                "bit_equal_to_baseline": bool(torch.equal(acc, accb)),
                                "rel_err_vs_oracle": fmt(np.linalg.norm(h - ref) / np.linalg.norm(ref)),
                                "norm_ratio": float(f"{float(acc.norm()) / float(X.norm()):.6e}")}
        del pl, prop, A
    return out


def bench_multi_rhs(torch, Plan, W, dev):
    """Random geometric graph, N = 2M, ~16 nnz/row, p = 6, k = 4..32, tile
    and group shapes picked by the autotuner."""
    import oracle as O
    from paper_2205_01598_amd import tune

    A, _ = W.random_geometric(2_000_000, 16.0, seed=0)
    out = {"workload": f"random geometric graph N=2M nnz={A.nnz}, row-normalised, p=6"}
    pl = Plan(A, 6, 256 << 20, root_mode=1)
    perm = pl.arrays()[0].astype(np.int64)
    for k in (4, 8, 16, 32):
        Xh = W.gaussian_block(A.n, k, seed=k)
        X = torch.from_numpy(np.ascontiguousarray(Xh[perm])).to(dev)
        Y = torch.empty((6, A.n, k), dtype=torch.float64, device=dev)
        pl.retune(6, 256 << 20, root_mode=1, nrhs=k)
        tb = timed(torch, lambda: pl.run_baseline(X, Y), 5, 2)
        Yb = Y.clone()
        cands = [dict(cache_mb=C, skew=s, tile_nnz=t) for C, s, t in
                 ((256, 2, 8192), (128, 2, 2048), (128, 3, 4096), (64, 3, 2048))]
        cfg, tm, _ = tune.autotune(torch, pl, 6, cands, lambda: pl.run(X, Y), nrhs=k)
        pl.run(X, Y)
        pl.status()
        ref = O.spmv_powers(A, Xh, 6, threads=oracle_threads())
        Yo = np.empty((6, A.n, k))
        Yo[:, perm] = Y.cpu().numpy()
        out[f"k{k}"] = {"mpk_ms": round(tm, 4), "baseline_ms": round(tb, 4), "speedup": round(tb / tm, 3),
                        "gflops": round(2.0 * A.nnz * 6 * k / tm / 1e6, 1), "config": cfg,
                        "max_rel_err_vs_oracle": fmt(max(rel_errs(Yo, ref))),
                        "bit_equal_to_baseline": bool(torch.equal(Y, Yb))}
        del X, Y, Yb, ref, Yo
    return out


def bench_thin_levels(torch, Plan, W, dev):
    """2D 9-point stencil on a 4096^2 grid (N = 16.8M, 151M nonzeros, 1.8 GB
    of FP64 CSR): 4096 levels of at most 4096 rows, so the level groups can
    be small and a large ticket skew keeps enough work in flight.  p = 8."""
    from paper_2205_01598_amd import tune

    A = W.stencil_2d(4096, 9)
    p = 8
    x = W.uniform_vector(A.n, seed=0)
    pl = Plan(A, p, 256 << 20, root_mode=1)
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    Y = torch.empty((p, A.n), dtype=torch.float64, device=dev)
    tb = timed(torch, lambda: pl.run_baseline(X, Y), 10, 2)
    ref = Y.clone()
    cands = [dict(cache_mb=C, skew=s, tile_nnz=t, workgroups=1024) for C, s, t in
             ((256, 2, 8192), (32, 12, 8192), (16, 24, 8192), (32, 8, 4096))]
    cfg, tm, timings = tune.autotune(torch, pl, p, cands, lambda: pl.run(X, Y), reps=10)
    runs = {f"C{c['cache_mb']}_s{c['skew']}_t{c['tile_nnz']}": round(t, 4) for c, t in timings}
    pl.run(X, Y)
    pl.status()
    flop = 2.0 * A.nnz * p
    import oracle as O

    Yo = np.empty((p, A.n))
    Yo[:, perm] = Y.cpu().numpy()
    err = fmt(max(rel_errs(Yo, O.spmv_powers(A, x, p, threads=oracle_threads()))))
    return {"workload": f"2D 9-point stencil 4096^2, n={A.n} nnz={A.nnz}, p={p}", "levels": pl.info()["n_levels"],
            "max_rel_err_vs_oracle": err,
            "level_groups": pl.info()["n_groups"], "mpk_ms": round(tm, 4), "baseline_ms": round(tb, 4),
            "speedup": round(tb / tm, 3), "gflops": round(flop / tm / 1e6, 1), "config": cfg,
            "bit_equal_to_baseline": bool(torch.equal(Y, ref)), "runs_ms": runs}


def probe():
    """Memory-hierarchy probes (the analog of the paper's Fig. 1, Sec. 2):
    load-only read rate against footprint for the L2 (4 MB per XCD), the
    256 MB Infinity Cache and HBM, with 1-8 loads in flight per thread and
    whole-buffer or per-XCD parts; the XCD placement of workgroups; and the
    latency of a flag hop between two workgroups at agent and at workgroup
    scope.  Prints a text report and one JSON line."""
    import torch

    from paper_2205_01598_amd import bw_probe
    from paper_2205_01598_amd.mpk import hop_probe, xcd_ids

    dev = torch.device("cuda:0")
    report = {}
    # ---- XCD placement ------------------------------------------------------------
    place = {}
    for wg, spin in ((64, 0), (1024, 0), (2048, 0), (1024, 2000), (2048, 2000), (8192, 200)):
        ids = torch.full((wg,), -1, dtype=torch.int32, device=dev)
        xcd_ids(ids, wg, spin)
        h = ids.cpu().numpy()
        exp = (h[0] + np.arange(wg)) % 8
        place[f"wg{wg}_spin{spin}"] = {"first_xcd": int(h[0]), "mismatch": int((h != exp).sum()),
                                       "per_xcd": np.bincount(h[h >= 0], minlength=8).tolist()}
    report["xcd_placement"] = place
    print(f"XCD placement (mismatches against (ids[0] + b) % 8): {place}", flush=True)
    # ---- flag hop latency ---------------------------------------------------------------
    flags = torch.zeros(64, dtype=torch.int32, device=dev)
    out = torch.zeros(2, dtype=torch.int64, device=dev)
    hops = {}
    for name, peer, scope in (("agent_scope_other_xcd", 1, 0), ("agent_scope_same_xcd", 8, 0),
                              ("workgroup_scope_same_xcd", 8, 1)):
        vals = []
        for _ in range(3):
            wall_khz = hop_probe(flags, peer, scope, 2000, 1 << 20, out)
            ticks, done = (int(t) for t in out.cpu().numpy())
            vals.append((ticks, done))
        best = min(t for t, d in vals if d == 2000) if all(d == 2000 for _, d in vals) else None
        hops[name] = {"one_way_ns": round(best / 4000 / wall_khz * 1e6, 1) if best else None,
                      "completed": [d for _, d in vals]}
    report["flag_hop"] = hops
    print(f"flag hop latency (one way): {hops}", flush=True)
    # ---- read rate against footprint ----------------------------------------------------
    buf = torch.empty(4 << 30, dtype=torch.uint8, device=dev).fill_(1)
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    modes = [("pass_u1_wg8192", 1, 8192, 1, False), ("pass_u4_wg2048", 4, 2048, 1, False),
             ("reread_u4_wg2048", 4, 2048, 1, True), ("reread_parts8_u4_wg2048", 4, 2048, 8, True),
             ("reread_parts8_u8_wg4096", 8, 4096, 8, True), ("reread_parts8_u2_wg8192", 2, 8192, 8, True)]
    rows = {}
    print("footprint_MB " + " ".join(f"{m[0]:>24s}" for m in modes) + "   (GB/s)", flush=True)
    for mb in (8, 16, 32, 48, 64, 96, 128, 160, 192, 256, 384, 512, 1024, 2048, 4096):
        b = buf[: mb << 20]
        line = {}
        for name, u, wg, parts, reread in modes:
            reps = max(1, (2048 // mb)) if reread else 1
            launches = 20 if not reread else 5
            t = timed(torch, lambda: bw_probe(b, reps, wg, sink, loads_per_thread=u, parts=parts), launches, 2)
            line[name] = round(reps * mb * (1 << 20) / t / 1e6, 1)
        rows[mb] = line
        print(f"{mb:10d} " + " ".join(f"{line[m[0]]:24.1f}" for m in modes), flush=True)
    report["read_GBps"] = rows
    print(json.dumps(report), flush=True)


def bench_learned_tuner(torch, plan, X, Y, p, log):
    """Train the cost model on the committed sweep database (held-out split),
    report its choices (alone, and its three best measured) against the
    sweep's best and the untuned default, and apply it to the headline
    matrix."""
    from paper_2205_01598_amd import tune

    db = os.path.join(ROOT, "paper_2205_01598_amd", "data", "tuner_sweep_mi355x.jsonl")
    if not os.path.exists(db):
        return None
    recs = tune.load_db(db)
    train, test = tune.split_seeds(recs)
    t0 = time.time()
    tuner = tune.LearnedTuner(hidden=64, seed=0)
    loss = tuner.fit(train, steps=6000)
    out = {"train_matrices": len({r["seed"] for r in train}), "held_out_matrices": len({r["seed"] for r in test}),
           "train_seconds": round(time.time() - t0, 2), "final_train_loss": round(loss, 5),
           "held_out": tune.evaluate(tuner, test, tune.best_static(train))}
    tune._apply(plan, p, tune.DEFAULT)
    feats = tune.plan_features(plan)
    t_def = tune.time_run(torch, plan, X, Y, reps=10)
    cfg = tuner.choose(feats)
    tune._apply(plan, p, cfg)
    t_pick = tune.time_run(torch, plan, X, Y, reps=10)
    # the model's three best configurations, measured (LearnedTuner.tune)
    cfg3, t3, _ = tuner.tune(torch, plan, p, lambda: plan.run(X, Y), m=3, reps=10)
    out["headline_matrix"] = {"chosen": cfg, "mpk_ms": round(t_pick, 4), "default_mpk_ms": round(t_def, 4),
                              "gain_over_default": round(t_def / t_pick, 3),
                              "shortlist3": {"chosen": cfg3, "mpk_ms": round(t3, 4),
                                             "gain_over_default": round(t_def / t3, 3)}}
    log(f"learned tuner: {out}")
    return out


def cpu_baseline_leg(A, x, p, flop):
    """The CPU oracle (plain C, FP64) timed on the same input, the way the
    paper runs its baseline (Sec. 6): the rows of every SpMV shared among all
    host threads this process may use (OpenMP, static schedule), and on one
    thread.  Both give the same result bit for bit; it is also the FP64
    reference of the GPU result."""
    import oracle as O

    threads = oracle_threads()
    runs, ref = [], None
    while sum(runs) < 10.0 and len(runs) < 40:
        t0 = time.time()
        ref = O.spmv_powers(A, x, p, threads=threads)
        runs.append(time.time() - t0)
    one = []
    while sum(one) < 10.0 and len(one) < 8:
        t0 = time.time()
        ref1 = O.spmv_powers(A, x, p)
        one.append(time.time() - t0)
    same = bool(np.array_equal(ref1, ref))
    del ref1
    cpu_s, one_s = float(np.mean(runs)), float(np.mean(one))
    cpu = {"value": round(flop / cpu_s / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(runs)} full FP64 p={p} runs (p back-to-back CSR SpMVs, rows shared among {threads} "
                     f"OpenMP threads, static schedule) of the same 160^3 matrix, mean {cpu_s:.3f} s "
                     f"(min {min(runs):.3f} s), on {cpu_model()} ({len(os.sched_getaffinity(0))} cores in the "
                     f"affinity mask)",
           "single_thread": {"value": round(flop / one_s / 1e9, 3), "cores": 1,
                             "sample": f"{len(one)} runs, mean {one_s:.2f} s (min {min(one):.2f} s)"},
           "threaded_equals_single_thread_bitwise": same}
    return cpu, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=160, help="grid edge of the 27-point matrix")
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the tuning sweep")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (2D 64^2, Chebyshev Anderson 128^3, multi-RHS RGG, "
                         "heat 160^3, learned tuner)")
    ap.add_argument("--only-main", action="store_true", help="only the headline p (no p=4/6)")
    ap.add_argument("--probe", action="store_true",
                    help="load-only bandwidth versus footprint (one full pass per launch) and exit")
    ap.add_argument("--thin-levels-only", action="store_true",
                    help="only the thin-level 2D 9-point 4096^2 workload (for profiling); prints its JSON and exits")
    ap.add_argument("--only-config", default=None, metavar="S_M,C_MB,SKEW,TILE,STREAMS",
                    help="only the headline matrix in this plan configuration (recursion stages, budget in MB, "
                         "skew, tile nonzeros, ticket streams): `steps` timed runs, one JSON line (for profiling)")
    ap.add_argument("--plan-device-only", action="store_true",
                    help="only planning the headline matrix from device memory (twice), one JSON line (for profiling)")
    args = ap.parse_args()
    if args.plan_device_only:
        plan_device_only(args)
        return
    if args.only_config:
        only_config(args)
        return
    if args.probe:
        probe()
        return
    if args.thin_levels_only:
        import torch

        import workloads as W
        from paper_2205_01598_amd import Plan

        print(json.dumps(bench_thin_levels(torch, Plan, W, torch.device("cuda:0"))), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2205_01598_amd import Plan, Spmv, tune

    dev = torch.device("cuda:0")
    p = args.p
    t0 = time.time()
    A, _ = W.stencil_27pt_random(args.n, seed=args.seed)
    x = W.uniform_vector(A.n, seed=args.seed)
    n, nnz = A.n, A.nnz
    log(f"generated 27-pt {args.n}^3: n={n} nnz={nnz} in {time.time() - t0:.1f}s")

    t0 = time.time()
    plan = Plan(A, p, 256 << 20, root_mode=1)
    plan_s = time.time() - t0
    perm = plan.arrays()[0].astype(np.int64)
    log(f"plan: {plan.info()['n_levels']} levels in {plan_s:.1f}s")
    # the same plan with the breadth-first levels on the GPU
    t0 = time.time()
    pdev = Plan(A, p, 256 << 20, root_mode=1, upload=False, plan_on_device=1)
    plan_dev_s = time.time() - t0
    assert np.array_equal(pdev.arrays()[0], plan.arrays()[0])
    plan_phases = {"host_levels": [round(v, 3) for v in plan.info()["phase_seconds"]],
                   "device_levels": [round(v, 3) for v in pdev.info()["phase_seconds"]]}
    del pdev
    log(f"plan with device levels: {plan_dev_s:.2f}s, phases {plan_phases}")
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    X0 = torch.from_numpy(x).to(dev)
    Y = torch.empty((p, n), dtype=torch.float64, device=dev)
    # the same plan from the CSR in device memory, which stays there (up to
    # a plan ready to run); its run equals the host plan's bit for bit
    dA = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (A.rowptr, A.col, A.val)]
    resident = {}
    pres = None
    for _ in range(2):
        del pres  # the previous plan is freed before the clock starts
        torch.cuda.synchronize()
        t0 = time.time()
        pres = Plan.from_device(*dA, p, 256 << 20, root_mode=1)
        torch.cuda.synchronize()
        resident["seconds"] = min(resident.get("seconds", 1e9), time.time() - t0)
    assert np.array_equal(pres.arrays()[0], plan.arrays()[0])
    Yr = torch.empty_like(Y)
    pres.run(X, Yr)
    plan.run(X, Y)
    pres.status()
    resident["bit_equal_to_host_plan_run"] = bool(torch.equal(Yr, Y))
    resident["phase_seconds"] = [round(v, 4) for v in pres.info()["phase_seconds"]]
    del pres, Yr, dA
    log(f"resident plan: {resident}")
    flop = 2.0 * nnz * p

    # ---- baselines: p back-to-back SpMV launches ------------------------------
    base = {}
    h = Spmv(A)
    base["given_order"] = timed(torch, lambda: h.powers(p, X0, Y), 5, 2)
    del h
    base["bfs_order"] = timed(torch, lambda: plan.run_baseline(X, Y), 10, 3)
    t_base = min(base.values())
    log(f"baselines (ms): {base}")

    # ---- MPK configuration: small sweep on the same levels ------------------------
    # tiles of 1, 2 and 3 whole 4096-nonzero chunks
    cands = [dict(cache_mb=256, skew=2, tile_nnz=8192), dict(cache_mb=256, skew=2, tile_nnz=12288),
             dict(cache_mb=256, skew=2, tile_nnz=4096), dict(cache_mb=512, skew=2, tile_nnz=8192)]
    if args.quick:
        cands = cands[:1]
    cfg, _, timings = tune.autotune(torch, plan, p, cands, lambda: plan.run(X, Y))
    for c, ms in timings:
        log(f"mpk {c}: {ms:.3f} ms")
    info = plan.info()

    # ---- calibration copy for the HBM counters: 256 MiB read + 256 MiB written ---------
    calib_src = torch.empty(32 << 20, dtype=torch.float64, device=dev).fill_(1.0)
    calib_dst = torch.empty_like(calib_src)
    calib_dst.copy_(calib_src)
    torch.cuda.synchronize()
    del calib_src, calib_dst

    # ---- timed region: exactly `steps` MPK runs ------------------------------------
    torch.cuda.synchronize()
    ms = timed(torch, lambda: plan.run(X, Y), args.steps, args.warmup)
    plan.status()
    Yh = np.empty((p, n))
    Yh[:, perm] = Y.cpu().numpy()
    gflops = flop / ms / 1e6
    alg_bytes = mpk_bytes(n, nnz, p)
    # per-call statistics over at least one second of single timed calls
    t_mean, t_min, t_med, t_n = timed_each(torch, lambda: plan.run(X, Y))
    plan.status()
    per_call = {"calls": t_n, "mean_ms": round(t_mean, 4), "min_ms": round(t_min, 4), "median_ms": round(t_med, 4)}
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    log(f"MPK p={p}: {ms:.3f} ms/step, {gflops:.1f} GFLOP/s, speedup {t_base / ms:.3f}")

    # ---- synchronisation ladder on the same plan: kernel boundary per Lp node, per
    # wavefront of independent nodes, then point-to-point flags (the timed MPK) ------
    G = info["n_groups"]
    ladder = {"level_groups": G, "launches": {"node": G * p, "wavefront": G + 2 * p - 2, "p2p_flags": 1},
              "launch_per_node_ms": round(timed(torch, lambda: plan.run_sync(X, Y, "node"), 3, 1), 4),
              "launch_per_wavefront_ms": round(timed(torch, lambda: plan.run_sync(X, Y, "wavefront"), 5, 1), 4),
              "p2p_flags_ms": round(ms, 4), "baseline_ms": round(t_base, 4)}
    # the persistent kernel's fixed cost: the same kernel with a budget that
    # puts every level in one group (no reuse window), then back to the pick
    plan.retune(p, 64 << 30, root_mode=1, skew=2, tile_nnz=int(cfg.get("tile_nnz", 8192)))
    ladder["one_level_group"] = {"groups": plan.info()["n_groups"],
                                 "ms": round(timed(torch, lambda: plan.run(X, Y), 10, 2), 4)}
    plan.status()
    tune.autotune(torch, plan, p, [cfg], lambda: plan.run(X, Y), reps=1, warmup=0)
    log(f"sync ladder: {ladder}")

    # ---- CPU oracle (FP64; all host threads and one) -----------------------------------
    ref = None
    cpu = None
    headline_parity = {}
    if not args.no_cpu:
        import oracle as O

        cpu, ref = cpu_baseline_leg(A, x, p, flop)
        errs = rel_errs(Yh, ref)
        log(f"cpu oracle {cpu['sample']}; MPK FP64 max rel err {max(errs):.2e}")
        # bit for bit: the oracle on the plan's renumbered matrix and input sums
        # every row in the kernel's order
        t0 = time.time()
        rp, pc, pv = O.permute_symmetric(A, perm)
        B_plan = W.CSR(n, rp, pc, pv)
        del rp, pc, pv
        xp = np.ascontiguousarray(x[perm])
        ref_plan = O.spmv_powers(B_plan, xp, p, threads=oracle_threads())
        plan_order_y = Y.cpu().numpy()
        headline_parity = {"max_rel_err_vs_oracle": fmt(max(errs)),
                           "bit_equal_to_oracle_on_plan_matrix": bool(np.array_equal(plan_order_y, ref_plan))}
        del ref_plan, plan_order_y
        log(f"plan-order oracle check in {time.time() - t0:.1f}s: {headline_parity}")

    # ---- recursive level refinement (Sec. 4.4) on the same matrix and launch options ----
    recursion = {"unrefined": {"ms": round(ms, 4), "level_groups": G, "violating_groups": info["violating_groups"]}}
    if not args.only_main:
        # at the headline's budget, then at the small budget where refinement
        # does best (level groups of at most about 1 MB), with one and with
        # eight XCD ticket streams
        for sm, cmb, streams in ((1, cfg["cache_mb"], 1), (2, cfg["cache_mb"], 1), (1, 20, 1), (1, 20, 8)):
            key = f"s_m={sm}" + ("" if cmb == cfg["cache_mb"] else f"_C{cmb}MB") + ("_xcd8" if streams == 8 else "")
            t0 = time.time()
            pr = Plan(A, p, cmb << 20, root_mode=1, skew=cfg["skew"], tile_nnz=cfg["tile_nnz"],
                      recursion_stages=sm, xcd_streams=streams)
            ps = time.time() - t0
            rperm = pr.arrays()[0].astype(np.int64)
            Xr = torch.from_numpy(np.ascontiguousarray(x[rperm])).to(dev)
            tr = timed(torch, lambda: pr.run(Xr, Y), 10, 2)
            pr.status()
            Yr = np.empty((p, n))
            Yr[:, rperm] = Y.cpu().numpy()
            ri = pr.info()
            recursion[key] = {"ms": round(tr, 4), "gflops": round(flop / tr / 1e6, 1),
                              "vs_unrefined": round(ms / tr, 3), "vs_baseline": round(t_base / tr, 3),
                              "units": ri["n_units"], "violating_groups": ri["violating_groups"],
                              "max_stage": ri["max_stage"], "dep_ranges_per_tile":
                              round(ri["n_dep_ranges"] / ri["n_tiles"], 2), "plan_seconds": round(ps, 2),
                              "max_rel_diff_vs_unrefined": float(f"{max(rel_errs(Yr, Yh)):.3e}")}
            if ref is not None:
                recursion[key]["max_rel_err_vs_oracle"] = fmt(max(rel_errs(Yr, ref)))
            del pr, Xr
        # bulky levels: the same matrix from an interior root (vertex 0 of the
        # random relabelling), and a power-law graph whose BFS levels are few
        # and fat (Zipf row lengths, exponent 2, uniform columns)
        for name, Aw, rm, pw in (("27pt160_interior_root", A, 0, p),
                                 ("zipf_4M_s2", W.zipf_rows(4_000_000, 2.0, seed=1), 1, 6)):
            xw = W.uniform_vector(Aw.n, seed=0)
            ent, ref_w = {}, None
            for sm in (0, 1):
                pw_plan = Plan(Aw, pw, 256 << 20, root_mode=rm, skew=2, tile_nnz=8192, recursion_stages=sm)
                wperm = pw_plan.arrays()[0].astype(np.int64)
                Xw = torch.from_numpy(np.ascontiguousarray(xw[wperm])).to(dev)
                Yw = torch.empty((pw, Aw.n), dtype=torch.float64, device=dev)
                if sm == 0:
                    ent["baseline_ms"] = round(timed(torch, lambda: pw_plan.run_baseline(Xw, Yw), 5, 2), 4)
                tw = timed(torch, lambda: pw_plan.run(Xw, Yw), 10, 2)
                pw_plan.status()
                Yr = np.empty((pw, Aw.n))
                Yr[:, wperm] = Yw.cpu().numpy()
                if ref_w is None:
                    import oracle as O

                    ref_w = ref if (Aw is A and ref is not None) else O.spmv_powers(Aw, xw, pw,
                                                                                    threads=oracle_threads())
                wi = pw_plan.info()
                ent[f"s_m={sm}"] = {"ms": round(tw, 4), "level_groups": wi["n_groups"],
                                    "violating_groups": wi["violating_groups"], "units": wi["n_units"],
                                    "max_rel_err_vs_oracle": fmt(max(rel_errs(Yr, ref_w)))}
                del pw_plan, Xw, Yw
            ent["workload"] = f"n={Aw.n} nnz={Aw.nnz} p={pw}"
            recursion[name] = ent
        log(f"recursion: {recursion}")

    # ---- other powers ----------------------------------------------------------------
    other = {}
    for q in (() if args.only_main else (4, 6)):
        if q == p:
            continue
        Yq = torch.empty((q, n), dtype=torch.float64, device=dev)
        plan.retune(q, 256 << 20, root_mode=1)
        tb = timed(torch, lambda: plan.run_baseline(X, Yq), 5, 2)
        cq, tq, _ = tune.autotune(torch, plan, q, cands, lambda: plan.run(X, Yq))
        other[f"p{q}"] = {"ms": round(tq, 4), "gflops": round(2.0 * nnz * q / tq / 1e6, 1),
                          "baseline_ms": round(tb, 4), "speedup": round(tb / tq, 3), "config": cq}
        if ref is not None:
            plan.run(X, Yq)
            plan.status()
            Yo = np.empty((q, n))
            Yo[:, perm] = Yq.cpu().numpy()
            other[f"p{q}"]["max_rel_err_vs_oracle"] = fmt(max(rel_errs(Yo, ref[:q])))
        del Yq

    # ---- mixed precision ------------------------------------------------------------
    mixed = {}
    if not args.no_mixed:
        # FP32 / BF16 storage with FP32 arithmetic (the default), and the same
        # storage with FP64 arithmetic ("_acc64": x read in FP64, products and
        # sums in FP64)
        for dt, acc in (("f32", 0), ("bf16", 0), ("f32", 1), ("bf16", 1)):
            pm = Plan(A, p, cfg["cache_mb"] << 20, root_mode=1, val_dtype=dt, accum_f64=acc, skew=cfg["skew"],
                      tile_nnz=cfg["tile_nnz"])
            tbm = timed(torch, lambda: pm.run_baseline(X, Y), 5, 2)
            Ybase = Y.clone()
            # the same small sweep as for FP64 (smaller values shift the best tile)
            mc = tune.autotune(torch, pm, p, cands + ([] if args.quick else
                                                      [dict(cache_mb=256, skew=2, tile_nnz=12288),
                                                       dict(cache_mb=256, skew=2, tile_nnz=16384)]),
                               lambda: pm.run(X, Y), val_dtype=dt, accum_f64=acc)[0]
            tm = timed(torch, lambda: pm.run(X, Y), 10, 3)
            pm.status()
            ent = {"ms": round(tm, 4), "gflops": round(flop / tm / 1e6, 1), "baseline_ms": round(tbm, 4),
                   "speedup": round(tbm / tm, 3), "speedup_vs_fp64_baseline": round(t_base / tm, 3),
                   "config": mc}
            pm.run(X, Y)
            pm.status()
            ent["bit_equal_to_baseline"] = bool(torch.equal(Y, Ybase))
            Ym = np.empty((p, n))
            Ym[:, perm] = Y.cpu().numpy()
            if ref is not None:
                # the stated error: against the FP64 oracle
                ent["rel_err_vs_fp64_oracle_per_power"] = [fmt(e) for e in rel_errs(Ym, ref)]
                # parity: the oracle's definition of this arithmetic on the
                # plan's matrix, bit for bit
                if acc:
                    dref = O.spmv_powers(O.round_values(B_plan, dt), xp, p, threads=oracle_threads())
                else:
                    dref = O.spmv_powers_lowp(B_plan, xp, p, dt)
                ent["bit_equal_to_oracle_definition"] = bool(np.array_equal(Y.cpu().numpy(), dref))
                del dref
            mixed[dt + ("_acc64" if acc else "")] = ent
            del pm, Ybase

    extra = {}
    if not args.no_extra:
        extra["learned_tuner"] = bench_learned_tuner(torch, plan, X, Y, p, log)
        del plan
        extra["small_2d"] = bench_small_2d(torch, Plan, W, dev)
        log(f"small 2D: {extra['small_2d']}")
        extra["chebyshev"] = bench_chebyshev(torch, Plan, W, dev)
        log(f"chebyshev: {extra['chebyshev']}")
        extra["multi_rhs"] = bench_multi_rhs(torch, Plan, W, dev)
        log(f"multi-RHS: {extra['multi_rhs']}")
        extra["heat"] = bench_heat(torch, Plan, W, dev)
        log(f"heat: {extra['heat']}")
        extra["thin_levels"] = bench_thin_levels(torch, Plan, W, dev)
        log(f"thin levels: {extra['thin_levels']}")

    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"27-point stencil {args.n}^3, random relabelling, FP64, single vector",
                   "n": n, "nnz": nnz, "p": p, "root": "pseudo-peripheral",
                   "cache_budget_mb": cfg["cache_mb"], "skew": cfg["skew"], "tile_nnz": cfg["tile_nnz"],
                   "workgroups": info["workgroups"], "levels": info["n_levels"],
                   "level_groups": info["n_groups"], "seed": args.seed},
        "speedup_vs_spmv": round(t_base / ms, 3),
        "per_call_timing": per_call,
        "baseline_ms": {k: round(v, 4) for k, v in base.items()},
        "baseline_gflops": round(flop / t_base / 1e6, 1),
        # the bytes p SpMVs move (matrix p times), per MPK time, and the
        # baseline's own rate: what the level blocking turns into speed
        "effective_GBps_as_p_spmvs": {"mpk": round(p * spmv_bytes(n, nnz) / (ms * 1e-3) / 1e9, 1),
                                      "baseline": round(p * spmv_bytes(n, nnz) / (t_base * 1e-3) / 1e9, 1)},
        "plan_seconds": round(plan_s, 2),
        "plan_spmv_equivalents": round(plan_s / (t_base / p * 1e-3), 0),
        "plan_seconds_plan_on_device": round(plan_dev_s, 2),
        "plan_device_resident": {"seconds": round(resident["seconds"], 4),
                                 "spmv_equivalents": round(resident["seconds"] / (t_base / p * 1e-3), 0),
                                 "phase_seconds": resident["phase_seconds"],
                                 "bit_equal_to_host_plan_run": resident["bit_equal_to_host_plan_run"]},
        "plan_phase_seconds": plan_phases,
        "sync_ladder": ladder,
        "recursion": recursion,
        "other_powers": other,
        "mixed_precision": mixed,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(),
                     "kernel": "mpk_persistent", "algorithmic_bytes": alg_bytes},
        "code_balance": code_balance(n, nnz, p),
        "cpu_baseline": cpu,
        "other_workloads": extra,
    }
    if ref is not None:
        out["fp64_max_rel_err"] = float(f"{max(rel_errs(Yh, ref)):.3e}")
        out["parity"] = headline_parity
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
