"""Benchmark of the hot path on one MI355X.

One step = the whole path over one batch of synthetic input: Parallel
Extraction (N starts x T Adam steps on the surrogate, rounding, exact
candidate, box test, pool, A g = 0 check, sort) -> minimality filter ->
multi-start augmentation from S feasible starts, with the instance's
kernel basis, starts and augmentation starts resident in HBM before the
timed region.

Workload (default): the QP-shaped instance, m = 20, n = 100 (d = 80),
A iid in {-1, 0, 1} with P(nonzero) = 0.3, nonconvex quadratic f with dense
symmetric Q ~ N(0, 1), bounds [-10, 10], 65536 starts x 2000 binary32
iterations on matrix cores, 200 augmentation starts (the paper's count).

Prints one JSON line (see the fields below).  The CPU baseline is the
oracle (plain binary64 numpy) timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3  # TFLOP/s, MI355X dense FP32 matrix
PEAK_BF16_MFMA = 2500.0  # TFLOP/s, MI355X dense bf16 matrix
PEAK_HBM = 8000.0       # GB/s
PEAK_FP32_VALU = 157.3  # TFLOP/s, MI355X fp32 vector (256 CUs x 4 SIMDs x 2.4 GHz, packed FMA)


def _big_kernel_name(stats, form):
    """The large-basis descent kernel an extraction ran, from its tile (or
    the sparse-form kernel, templated on the 64-coordinate slots per lane)."""
    if stats.get("row_entries", 0) > 0:
        return f"k_descent_sparse<{_sparse_dc(stats['d'])}>" if "d" in stats else "k_descent_sparse"
    return f"k_descent_big<{stats.get('tile_slices', 0)},{stats.get('tile_blocks', 0)},{form}>"


def _sparse_dc(d):
    """Coordinate slots of 64 per lane of the sparse-form kernel instance for d."""
    return next(c for c in (2, 4, 6, 8, 12, 16) if 64 * c >= d)


def sparse_roofline(nnz, d, N, T, ms):
    """Roofline of one sparse-form descent launch (ALU bound).  Algorithmic
    work per start-iteration: 2 flop per nonzero of B for the forward B z, 1
    (a signed integer add) per nonzero for the backward B^T sign(B z), and 20
    per coordinate for the integrality and barrier terms and Adam (term 7,
    first moment 3, second moment 4, step 6); priced at the fp32 vector peak."""
    ops = (3.0 * nnz + 20.0 * d) * N * T
    t = ms * 1e-3
    return {"achieved": ops / t / 1e12, "peak": PEAK_FP32_VALU, "frac": ops / t / 1e12 / PEAK_FP32_VALU,
            "algorithmic": "3*nnz(B) + 20*d flop per start-iteration (forward multiply-adds, backward signed adds, "
                           "Adam and the integrality term per coordinate)"}


def descent_roofline(n, d, N, T, ms, bf16_iters=0):
    """Roofline of one descent launch.  Algorithmic work: 4 n d flop per
    start-iteration, 2 n d for the forward B z and 2 n d for the backward
    B^T sign(B z).  Each product is priced at the peak of the matrix unit it
    runs on: the backward on bf16 (exact operands) in every mode, the forward
    on FP32 except in the bf16 iterations.  `peak` is the resulting
    time-weighted peak (work / time at peak), `frac` the time at peak over the
    measured time."""
    half = 2.0 * n * d * N
    polish = T - bf16_iters
    t_peak = (polish * (half / PEAK_FP32_MFMA + half / PEAK_BF16_MFMA) +
              bf16_iters * 2.0 * half / PEAK_BF16_MFMA) / 1e12
    flops = 2.0 * half * T
    t = ms * 1e-3
    return {"achieved": flops / t / 1e12, "peak": flops / t_peak / 1e12, "frac": t_peak / t,
            "peak_note": "time-weighted: forward at the FP32 matrix peak 157.3 TFLOP/s "
                         f"({polish} binary32 iterations) or bf16 2500 TFLOP/s ({bf16_iters} bf16 iterations), "
                         "backward at the bf16 peak 2500 TFLOP/s"}

# HBM traffic of the descent kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a copy of known
# size.  The summary records a hash of the kernel's sources; a figure taken
# on other sources is not reported.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_descent_f32_qp_m20_n100_hbm_traffic.md")
KERNEL_SOURCES = ["paper_2412_13576_amd/csrc/descent_f32.hip", "paper_2412_13576_amd/csrc/graver_internal.h",
                  "paper_2412_13576_amd/csrc/pool_device.h"]
TRAFFIC_PROFILE_BIG = os.path.join(ROOT, "profiles", "k_descent_big_quartic_m50_n400_hbm_traffic.md")
KERNEL_SOURCES_BIG = ["paper_2412_13576_amd/csrc/descent_big.hip", "paper_2412_13576_amd/csrc/graver_internal.h"]
TRAFFIC_PROFILE_SPARSE = os.path.join(ROOT, "profiles", "k_descent_sparse_quartic_m50_n400_hbm_traffic.md")
KERNEL_SOURCES_SPARSE = ["paper_2412_13576_amd/csrc/descent_sparse.hip", "paper_2412_13576_amd/csrc/descent_sparse.h",
                         "paper_2412_13576_amd/csrc/graver_internal.h"]


def kernel_sources_sha256(sources=None) -> str:
    h = hashlib.sha256()
    for rel in (sources or KERNEL_SOURCES):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _measured_traffic(N, T, precision, profile=None, sources=None):
    """Bytes per descent launch recorded for these sources and this launch
    shape, or None."""
    profile = profile or TRAFFIC_PROFILE
    try:
        with open(profile) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith(("#", "|", "`")))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_sources_sha256(sources):
        return None
    if kv.get("launch") != f"N={N} T={T} {precision}":
        return None
    return float(kv["hbm_bytes_per_launch"])


def _oracle_extract(A, B, P, l, u, seed, n_sample, T):
    """One oracle extraction (Algorithm 2 in binary64 numpy) on n_sample box
    starts, with numpy's BLAS held to one thread; returns its seconds."""
    from threadpoolctl import threadpool_limits

    from oracle import philox
    from oracle import surrogate as S
    _, z0 = philox.box_starts(P, l, u, n_sample, seed=seed)
    with threadpool_limits(1):
        t = time.perf_counter()
        S.extract(A, B, l, u, z0, T, S.AdamParams(), check_kernel=False)
        return time.perf_counter() - t


def _oracle_worker(args, barrier, out):
    """Process body of the all-cores baseline: wait for every worker, then time
    one extraction."""
    barrier.wait()
    out.put(_oracle_extract(*args))


def _cpu_baseline(inst, T, n_sample=512):
    """The oracle on the host cores, on a bounded sample of the workload
    (n_sample starts per process, T iterations): one process, then one
    process per core started together.  Runs before this process touches the
    GPU, so the worker processes are plain interpreters.  start-iterations/s."""
    import multiprocessing as mp

    from oracle import lattice
    B = lattice.kernel_basis(inst.A)
    P = lattice.coordinate_projector(B)
    single = _oracle_extract(inst.A, B, P, inst.l, inst.u, 99, n_sample, T)
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(procs + 1)
    out = ctx.Queue()
    workers = [ctx.Process(target=_oracle_worker,
                           args=((inst.A, B, P, inst.l, inst.u, 100 + i, n_sample, T), barrier, out))
               for i in range(procs)]
    single_only = {"value": n_sample * T / single, "unit": "start-iterations/s", "cores": 1, "kind": "oracle",
                   "sample": f"{n_sample} starts x {T} iterations of the same instance (binary64 numpy, one "
                             f"process, one BLAS thread), {single:.1f} s"}
    for w in workers:
        w.start()
    try:
        barrier.wait(timeout=300)
        t = time.perf_counter()
        secs = [out.get(timeout=600) for _ in workers]
        wall = time.perf_counter() - t
    except Exception as exc:  # a worker did not start or finish: report the one-process figure
        for w in workers:
            w.terminate()
        print(f"[bench] all-cores oracle baseline skipped: {exc!r}", file=sys.stderr, flush=True)
        return single_only
    for w in workers:
        w.join(timeout=60)
    return {"value": procs * n_sample * T / wall, "unit": "start-iterations/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} processes x {n_sample} starts x {T} iterations of the same instance (binary64 "
                      f"numpy, one BLAS thread per process), {wall:.1f} s wall (slowest process {max(secs):.1f} s)",
            "single_core": {"value": n_sample * T / single, "cores": 1,
                            "sample": f"{n_sample} starts x {T} iterations, one process, one BLAS thread, "
                                      f"{single:.1f} s"}}


def _bases(insts, lll):
    """Host kernel bases of many instances on a thread pool (ctypes releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2412_13576_amd import graver as G
    with ThreadPoolExecutor(max_workers=16) as ex:
        return list(ex.map(lambda it: G.kernel_basis(it[0].A, lll=it[1]), [(i, l) for i, l in zip(insts, lll)]))


def _copy_calibration():
    """One device-to-device copy of 1 GiB: a dispatch whose HBM bytes are
    known, run in the profiled process to scale the FETCH_SIZE / WRITE_SIZE
    counters of the other dispatches."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _line(metric, value, unit, steps, warmup, ms, dtype, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_precision(args):
    """The precision comparison: quartic workload (m=50, n=400, d=350),
    262144 starts x 2000 iterations, binary32 vs bf16 (+10% binary32
    polish); extraction throughput at full size, recall of the filtered
    sets against filter(F_fp32 u F_bf16) at 65536 starts."""
    import torch

    from paper_2412_13576_amd import graver as G
    from paper_2412_13576_amd import workloads as W
    inst = W.quartic_instance()
    B, P = G.kernel_basis(inst.A)
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    N, T = args.starts or 262144, args.iters
    res = {}
    for prec in ("fp32", "bf16"):
        pv = G.GRAVER_FP32 if prec == "fp32" else G.GRAVER_BF16
        # (both forms on matrix cores: the comparison is between the binary32
        # and the bf16 contractions)
        fm = G.GRAVER_FORM_DENSE
        prm = G.extract_params(N, T, precision=pv, init_mode=0, seed=3, polish_iters=T // 10 if prec == "bf16" else 0,
                               collect=0, form=fm)
        G.extract(ctx, prob, G.extract_params(4096, 8, precision=pv, init_mode=0, seed=1, collect=0, form=fm))
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = G.extract(ctx, prob, prm)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        res[prec] = {"descent_ms": st["ms_descent"], "wall_ms": el * 1e3, "kernel": _big_kernel_name(st, prec),
                     "start_iterations_per_s": N * T / el,
                     "tflops": 4.0 * inst.n * B.shape[1] * N * T / (st["ms_descent"] * 1e-3) / 1e12}
        print(f"[precision] {prec} descent {st['ms_descent']:.1f} ms", file=sys.stderr, flush=True)
    # recall at 65536 starts (the full-size sets hold ~1e8 keys of 400 bytes)
    Nr = min(N, 65536)
    F = {}
    for prec in ("fp32", "bf16"):
        pv = G.GRAVER_FP32 if prec == "fp32" else G.GRAVER_BF16
        k, st = G.extract(ctx, prob, G.extract_params(Nr, T, precision=pv, init_mode=0, seed=3, pool_capacity=1 << 25,
                                                      polish_iters=T // 10 if prec == "bf16" else 0,
                                                      form=G.GRAVER_FORM_DENSE))
        F[prec] = G.filter_minimal(ctx, k)
        res[prec]["unique_at_recall_size"] = int(k.shape[0])
        del k
        print(f"[precision] {prec} filtered {F[prec].shape[0]}", file=sys.stderr, flush=True)
    ref = G.filter_minimal(ctx, torch.cat([F["fp32"], F["bf16"]]))
    rv = np.ascontiguousarray(ref.cpu().numpy()).view(np.dtype((np.void, ref.shape[1]))).ravel()
    for prec in ("fp32", "bf16"):
        fv = np.ascontiguousarray(F[prec].cpu().numpy()).view(np.dtype((np.void, ref.shape[1]))).ravel()
        res[prec]["recall"] = float(np.isin(rv, fv).sum() / max(1, rv.size))
    n_, d_ = inst.n, B.shape[1]
    roof32 = descent_roofline(n_, d_, N, T, res["fp32"]["descent_ms"])
    rb = descent_roofline(n_, d_, N, T, res["bf16"]["descent_ms"], bf16_iters=T - T // 10)
    res["bf16"]["roofline"] = {k: rb[k] for k in ("achieved", "peak", "frac")}
    _line("start-iterations/s of the descent, bf16 vs binary32 (extraction, precision comparison)",
          res["bf16"]["start_iterations_per_s"], "start-iterations/s", 1, 1, res["bf16"]["wall_ms"], "bf16+f32",
          {"workload": "quartic_m50_n400: m=50, n=400 (d=350), 4 nonzeros per row in +-1..+-5, separable "
                       "quartic f, box [-20,20]", "starts": N, "iters": T, "recall_starts": Nr,
           "forms": "both on matrix cores (the binary32 default on this basis is the sparse form)"},
          precision=res, speedup_bf16_over_fp32=res["fp32"]["wall_ms"] / res["bf16"]["wall_ms"],
          roofline={"bound": "mfma", "kernel": res["fp32"]["kernel"], "achieved": roof32["achieved"],
                    "peak": roof32["peak"], "unit": "TFLOP/s", "frac": roof32["frac"], "traffic": None,
                    "peak_note": roof32["peak_note"],
                    "note": "binary32 launch; the bf16 launch is reported in precision.bf16.roofline"})
    ctx.close()


def bench_batch(args):
    """Batching: 64 instances, n uniform in [50, 500], m = round(U(0.1, 0.3) n),
    A iid (0 w.p. 0.8, else +-1, +-2), box [-5, 5], 256 n starts each, 1000
    iterations, one batched extraction (autotuned tiles, graph-captured
    rounds), bf16 vs binary32; against the same instances extracted one call
    at a time.  Host kernel bases (not timed) are reported beside."""
    import torch

    from paper_2412_13576_amd import graver as G
    from paper_2412_13576_amd import workloads as W
    rng = np.random.default_rng(4000)
    ns = rng.integers(50, 501, size=64)
    ms = [int(round(rng.uniform(0.1, 0.3) * n)) for n in ns]
    insts = [W.sparse_quadratic_instance(4000 + k, int(n), m) for k, (n, m) in enumerate(zip(ns, ms))]
    t_b = time.perf_counter()
    bases = _bases(insts, [True] * len(insts))
    basis_s = time.perf_counter() - t_b
    print(f"[batch] host bases {basis_s:.1f} s", file=sys.stderr, flush=True)
    T = args.iters if args.iters != 2000 else 1000
    probs = [G.DeviceProblem.from_numpy(it.A, it.b, it.l, it.u, B, P) for it, (B, P) in zip(insts, bases)]
    Ns = [256 * it.n for it in insts]
    caps = [int(N * max(8, 6000 // it.n)) for N, it in zip(Ns, insts)]
    total = sum(Ns) * T
    ctx = G.Context(0)
    res = {}
    for prec in ("fp32", "bf16"):
        pv = G.GRAVER_FP32 if prec == "fp32" else G.GRAVER_BF16
        prms = [G.extract_params(N, T, precision=pv, init_mode=0, seed=k, pool_capacity=c,
                                 polish_iters=T // 10 if prec == "bf16" else 0) for k, (N, c) in enumerate(zip(Ns, caps))]
        # warmup with every instance at full size and 8 iterations: loads the
        # code objects and runs the tile-shape trials, which the context keeps
        G.extract_batch(ctx, probs, [G.extract_params(N, 8, precision=pv, init_mode=0, seed=1, pool_capacity=c)
                                     for N, c in zip(Ns, caps)], autotune=True, use_graph=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        keys, stats, bs = G.extract_batch(ctx, probs, prms, autotune=True, use_graph=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        res[prec] = {"wall_ms": el * 1e3, "start_iterations_per_s": total / el, "batched_descent_ms": bs["ms_descent"],
                     "launches": bs["launches"], "graphs": bs["graphs"], "replays": bs["replays"],
                     "unique": int(sum(s["unique"] for s in stats))}
        del keys
        print(f"[batch] {prec} {el * 1e3:.0f} ms", file=sys.stderr, flush=True)
    # the same binary32 work one instance per call
    prms = [G.extract_params(N, T, precision=G.GRAVER_FP32, init_mode=0, seed=k, pool_capacity=c)
            for k, (N, c) in enumerate(zip(Ns, caps))]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for p, pr, c in zip(probs, prms, caps):
        G.extract(ctx, p, pr, keys_cap=c)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t
    res["fp32_one_call_per_instance"] = {"wall_ms": seq * 1e3, "start_iterations_per_s": total / seq}
    _line("start-iterations/s, 64 instances in one batched extraction (bf16)", res["bf16"]["start_iterations_per_s"],
          "start-iterations/s", 1, 1, res["bf16"]["wall_ms"], "bf16+f32",
          {"workload": "64 instances, n ~ U{50..500}, m = round(U(0.1,0.3) n), A iid density 0.2 in "
                       "+-1,+-2, box [-5,5], quadratic f", "starts": "256 n per instance", "iters": T,
           "total_start_iterations": total}, batch=res, host_basis_s=basis_s)
    ctx.close()


def _serve_run(R, n_max=1000, rate=50.0, seed=5000):
    """R Poisson arrivals at `rate`/s, n log-uniform in [20, n_max], m =
    round(0.2 n), A iid (0 w.p. 0.8, else +-1, +-2), quadratic (box [-5,5])
    or separable quartic objective (box [-20,20]) 50/50, binary32 or bf16
    descent 50/50, 16 n starts x 500 iterations, 8 initial-solution starts
    plus the instance's feasible point.  Returns the measured figures."""
    from paper_2412_13576_amd import graver as G
    from paper_2412_13576_amd import workloads as W
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(np.log(20), np.log(n_max), size=R)).astype(int)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=R))
    reqs = []
    for k, n in enumerate(ns):
        m = max(1, int(round(0.2 * n)))
        inst = W.sparse_quadratic_instance(seed + k, int(n), m)
        N = 16 * int(n)
        bf = rng.random() < 0.5
        ex = G.extract_params(N, 500, precision=G.GRAVER_BF16 if bf else G.GRAVER_FP32, init_mode=0, seed=k,
                              pool_capacity=int(N * max(8, 3000 // int(n))), polish_iters=50 if bf else 0)
        ini = G.init_params(8, 200, seed=k + 1, lr=0.05)
        l, u = inst.l, inst.u
        if rng.random() < 0.5:
            obj = dict(Q=inst.Q, c=inst.c)
        else:
            l, u = np.full(int(n), -20, np.int64), np.full(int(n), 20, np.int64)  # the quartic law's box
            coef = np.zeros((int(n), 5))
            coef[:, 4] = rng.uniform(0.1, 1.0, int(n))
            coef[:, 3] = rng.standard_normal(int(n))
            coef[:, 2] = rng.standard_normal(int(n))
            obj = dict(coef=coef)
        reqs.append((inst, l, u, ex, ini, obj, N))
    srv = G.Server(hbm_budget=200 << 30, max_batch=32, gpu_workers=2, host_threads=16, autotune=False,
                   use_graph=True, batch_window_us=2000)
    t0 = time.perf_counter()
    tickets = []
    for (inst, l, u, ex, ini, obj, N), at in zip(reqs, arrivals):
        dt = at - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(inst.A, inst.b, l, u, ex, ini, lll=True, x_starts=inst.x0[None, :], **obj))
    results = [srv.wait(t)[0] for t in tickets]
    el = time.perf_counter() - t0
    srv.close()
    ok = [r for r in results if r["status"] == 0]
    lat = np.array([r["t_done"] - r["t_submit"] for r in ok]) * 1e3
    queue = np.array([r["t_admit"] - r["t_ready"] for r in ok]) * 1e3
    prep = np.array([r["t_ready"] - r["t_submit"] for r in ok]) * 1e3
    gpu = np.array([r["t_done"] - r["t_admit"] for r in ok]) * 1e3
    pct = lambda x: {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99))}
    iters = sum(N * 500 for (*_, N), r in zip(reqs, results) if r["status"] == 0)
    return {"requests": R, "rate_per_s": rate, "n_range": [20, n_max], "wall_s": el, "completed_per_s": len(ok) / el,
            "failed": len(results) - len(ok), "latency_ms": dict(pct(lat), max=float(lat.max())),
            "basis_ms": pct(prep), "queue_ms": pct(queue), "gpu_ms": pct(gpu),
            "start_iterations_per_s": iters / el, "mean_batch_size": float(np.mean([r["batch_size"] for r in ok]))}


def bench_serve(args):
    """Serving: the request stream of _serve_run at 50 requests/s, n up to --n-max."""
    R = args.requests
    r = _serve_run(R, n_max=args.n_max)
    _line("requests/s at Poisson 50 req/s arrivals (p50/p99 solve latency beside)", r["completed_per_s"],
          "requests/s", R, 0, r["wall_s"] * 1e3 / R, "f32|bf16",
          {"workload": f"Poisson 50/s, n log-uniform [20,{args.n_max}], m = round(0.2 n), A iid density 0.2 in +-1,+-2, "
                       "quadratic (box [-5,5]) or quartic (box [-20,20]), fp32 or bf16, 16 n starts x 500 "
                       "iterations", "requests": R}, **{k: v for k, v in r.items() if k not in ("requests",)})


def bench_augment(args):
    """Multi-start augmentation (Algorithm 1 from every start) on the QP
    workload with a direction set short enough to move interior points: the
    filtered binary32 extraction from Gaussian coordinate starts (sigma 0.5),
    then 200 feasible-walk starts.  (With the box-uniform starts of the main
    benchmark the extracted directions sit at the edge of the box and no
    start can move.)  Reports (direction, start) evaluations per second."""
    import torch

    from paper_2412_13576_amd import graver as G
    from paper_2412_13576_amd import workloads as W
    inst = W.qp_instance(2000)
    B, P = G.kernel_basis(inst.A)
    n, d = B.shape
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    obj = G.objective("quadratic", Q=inst.Q, c=inst.c)
    N, T = args.starts or 16384, args.iters
    z0 = torch.tensor(W.gaussian_starts(N, d, 0.5, 5), device="cuda")
    prm = G.extract_params(N, T, precision=G.GRAVER_FP32, init_mode=1, pool_capacity=1 << 23, any_order=True)
    keys, _ = G.extract(ctx, prob, prm, state={"z": z0})
    F = G.filter_minimal(ctx, keys)
    del keys
    S0 = args.aug_starts
    starts = torch.tensor(W.feasible_walk_starts(inst.x0, B.T.copy(), inst.l, inst.u, S0, seed=7, walk_len=32),
                          device="cuda")
    print(f"[augment] {F.shape[0]} directions, {S0} starts", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        G.augment(ctx, prob, obj, F, starts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        x, f, steps, best = G.augment(ctx, prob, obj, F, starts)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / args.steps
    st = steps.cpu().numpy()
    K = int(F.shape[0])
    pairs = K * float((st + 1).sum())  # every active start scores every direction once per pass
    nnz = float((F != 0).sum(dim=1).double().mean().item())
    f0 = G.augment(ctx, prob, obj, F[:0], starts)[1].cpu().numpy()
    _line("(direction, start) evaluations/s of the augmentation (Algorithm 1 from every start)", pairs / el,
          "evaluations/s", args.steps, args.warmup, el * 1e3, "f64",
          {"workload": "qp_m20_n100 augmentation: directions = filtered binary32 extraction from "
                       f"{N} Gaussian coordinate starts (sigma 0.5) x {T} iterations; {S0} feasible-walk starts",
           "directions": K, "aug_starts": S0},
          mean_nnz_per_direction=nnz, steps_total=int(st.sum()), steps_max=int(st.max()), passes=int(st.max()) + 1,
          f_start_mean=float(f0.mean()), f_end_mean=float(f.cpu().numpy().mean()), best_f=float(f[best].item()),
          f64_flop_lower_bound_tflops=2.0 * nnz * pairs / el / 1e12)
    ctx.close()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_quartic(args):
    """The whole path on the largest single-GPU configuration: the quartic
    workload (m = 50, n = 400, d = 350, 4 nonzeros per row in +-1..+-5,
    separable degree-4 f, box [-20, 20]), 262144 box starts x 2000 binary32
    iterations per step: Parallel Extraction with collection (about 9.5e7
    distinct verified candidates), the minimality filter over all of them,
    and the augmentation from 200 feasible starts.  The filter's two
    key-sized buffers take the slots of the extraction's pool and log, so the
    stages fit in device memory together and the workspace, allocated in the
    warmup step, is reused by every timed step.  Beside: one step with the
    bf16 form (exact three-part bf16 forward, last 10% binary32 polish) and a
    short serving leg."""
    from paper_2412_13576_amd import workloads as W

    inst = W.quartic_instance()
    N, T, S0 = args.starts or 262144, args.iters, args.aug_starts
    # the host baseline runs first, before anything here touches the GPU; the
    # sample is bounded (64 starts x 1000 iterations per process)
    cpu = None if args.no_cpu_baseline else _cpu_baseline(inst, min(T, 1000), n_sample=64)

    import torch

    from paper_2412_13576_amd import graver as G

    B, P = G.kernel_basis(inst.A)              # host C++ (Lemma 3.1 + LLL), not timed
    n, d = B.shape
    Bp = np.zeros(((n + 15) // 16 * 16, (d + 15) // 16 * 16), dtype=np.int64)
    Bp[:n, :d] = B
    blocks = (Bp.reshape(Bp.shape[0] // 16, 16, Bp.shape[1] // 16, 16) != 0).any(axis=(1, 3))
    nzb, nb_total = int(blocks.sum()), int(blocks.size)
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    obj = G.objective("separable_poly", coef=inst.coef)
    starts = torch.tensor(W.feasible_walk_starts(inst.x0, B.T.copy(), inst.l, inst.u, S0, seed=7, walk_len=32),
                          device="cuda")
    pool_cap = max(1 << 22, 500 * N)

    def step(seed, prec):
        polish = T // 10 if prec == G.GRAVER_BF16 else 0
        prm = G.extract_params(N, T, precision=prec, init_mode=0, seed=seed, pool_capacity=pool_cap,
                               polish_iters=polish, any_order=True)  # the filter sorts
        t0 = time.perf_counter()
        keys, st = G.extract(ctx, prob, prm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        F = G.filter_minimal(ctx, keys)
        K = int(keys.shape[0])
        del keys
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        x, f, steps, best = G.augment(ctx, prob, obj, F, starts)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        rec = dict(unique=K, filtered=int(F.shape[0]), stats=st, t_extract=t1 - t0, t_filter=t2 - t1,
                   t_augment=t3 - t2, best_f=float(f[best].item()), mean_steps=float(steps.double().mean().item()))
        del F
        return rec

    for w in range(args.warmup):
        step(1000 + w, G.GRAVER_FP32)
        print(f"[quartic] warmup step {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for k in range(args.steps):
        recs.append(step(2000 + k, G.GRAVER_FP32))
        print(f"[quartic] step {k}: {recs[-1]['t_extract']:.2f} + {recs[-1]['t_filter']:.2f} + "
              f"{recs[-1]['t_augment']:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el * 1000.0 / args.steps
    desc_ms = float(np.mean([r["stats"]["ms_descent"] for r in recs]))
    nnz = int(np.count_nonzero(B))
    st_last = dict(recs[-1]["stats"], d=d)
    sparse_form = st_last["row_entries"] > 0
    if sparse_form:
        roof = sparse_roofline(nnz, d, N, T, desc_ms)
        roofline = {"bound": "alu", "kernel": _big_kernel_name(st_last, "fp32"), "achieved": roof["achieved"],
                    "peak": roof["peak"], "unit": "TFLOP/s", "frac": roof["frac"],
                    "traffic": _measured_traffic(N, T, "fp32", TRAFFIC_PROFILE_SPARSE, KERNEL_SOURCES_SPARSE),
                    "algorithmic": roof["algorithmic"],
                    "peak_note": "fp32 vector peak; the kernel's limits are LDS and VALU instruction issue (gathers "
                                 "and integer scatter-adds over B's row lists), one start per wavefront",
                    "note": f"sparse form: B has {nnz} nonzeros of {n * d} ({st_last['row_entries']} row-list "
                            "entries per lane); the matrix-core kernel on the same launch is in dense_form"}
    else:
        roof = descent_roofline(n, d, N, T, desc_ms)
        roofline = {"bound": "mfma", "kernel": _big_kernel_name(st_last, "fp32"), "achieved": roof["achieved"],
                    "peak": roof["peak"], "unit": "TFLOP/s", "frac": roof["frac"],
                    "traffic": _measured_traffic(N, T, "fp32", TRAFFIC_PROFILE_BIG, KERNEL_SOURCES_BIG),
                    "algorithmic": "4*n*d flop per start-iteration (B z forward + B^T sign backward)",
                    "peak_note": roof["peak_note"],
                    "note": "algorithmic work is counted dense; the binary32 kernel skips the products of the zero "
                            f"16x16 blocks of B ({nzb} of {nb_total} blocks are nonzero here)"}
    mean = lambda key: float(np.mean([r[key] for r in recs]))
    out = {
        "metric": "start-iterations/s (whole path: extraction + filter + augmentation)",
        "value": N * T * args.steps / el,
        "unit": "start-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "quartic_m50_n400: m=50, n=400 (d=350), A with 4 nonzeros per row in +-1..+-5, "
                               "separable degree-4 f, box [-20,20] (the precision configuration's instance, binary32 "
                               "form)", "starts": N, "iters": T, "aug_starts": S0,
                   "precision": "fp32-sparse" if sparse_form else "fp32-mfma"},
        "verified_directions_per_s": mean("unique") / (ms_step * 1e-3),
        "verified_directions_per_s_extraction": mean("unique") / mean("t_extract"),
        "descent_start_iterations_per_s": N * T / (desc_ms * 1e-3),
        "stage_s": {"extract": mean("t_extract"), "filter": mean("t_filter"), "augment": mean("t_augment")},
        "extract": {k: float(np.mean([r["stats"][k] for r in recs])) for k in
                    ("emit_events", "inbox_events", "unique", "verified", "out_of_range",
                     "ms_init", "ms_descent", "ms_verify", "ms_sort")},
        "filtered": mean("filtered"),
        "aug_best_f": recs[-1]["best_f"],
        "aug_mean_steps": recs[-1]["mean_steps"],
        "roofline": roofline,
    }
    if sparse_form and not args.no_dense_leg:
        # the binary32 matrix-core kernel on the same launch (extraction only)
        torch.cuda.synchronize()
        prm = G.extract_params(N, T, precision=G.GRAVER_FP32, init_mode=0, seed=2000, pool_capacity=pool_cap,
                               any_order=True, form=G.GRAVER_FORM_DENSE)
        kd, sd = G.extract(ctx, prob, prm)
        del kd
        torch.cuda.synchronize()
        rd = descent_roofline(n, d, N, T, sd["ms_descent"])
        out["dense_form"] = {
            "kernel": _big_kernel_name(dict(sd, d=d), "fp32"), "descent_ms": sd["ms_descent"],
            "unique": sd["unique"], "sparse_speedup": sd["ms_descent"] / desc_ms,
            "roofline": {"bound": "mfma", "achieved": rd["achieved"], "peak": rd["peak"], "frac": rd["frac"],
                         "unit": "TFLOP/s", "algorithmic": "4*n*d flop per start-iteration",
                         "traffic": _measured_traffic(N, T, "fp32", TRAFFIC_PROFILE_BIG, KERNEL_SOURCES_BIG),
                         "note": f"dense count; the kernel skips the zero 16x16 blocks of B ({nzb} of {nb_total} "
                                 "are nonzero)"}}
        print(f"[quartic] dense-form descent {sd['ms_descent']:.0f} ms", file=sys.stderr, flush=True)
    if not args.no_bf16_line:
        torch.cuda.synchronize()
        tb = time.perf_counter()
        rb = step(3000, G.GRAVER_BF16)
        torch.cuda.synchronize()
        elb = time.perf_counter() - tb
        rfb = descent_roofline(n, d, N, T, rb["stats"]["ms_descent"], bf16_iters=T - T // 10)
        out["bf16_polish"] = {
            "start_iterations_per_s": N * T / elb, "ms_per_step": elb * 1e3,
            "descent_ms": rb["stats"]["ms_descent"], "unique": rb["unique"], "filtered": rb["filtered"],
            "stage_s": {"extract": rb["t_extract"], "filter": rb["t_filter"], "augment": rb["t_augment"]},
            "speedup_descent_over_fp32": desc_ms / rb["stats"]["ms_descent"],
            "speedup_descent_over_fp32_matrix_cores": (out["dense_form"]["descent_ms"] / rb["stats"]["ms_descent"]
                                                       if "dense_form" in out else desc_ms / rb["stats"]["ms_descent"]),
            "roofline": {"achieved": rfb["achieved"], "peak": rfb["peak"], "frac": rfb["frac"], "unit": "TFLOP/s"},
            "form": "forward on bf16 matrix cores with z split exactly into three bf16 parts, fp32 accumulation; "
                    f"last {T // 10} iterations binary32"}
        print(f"[quartic] bf16 step {elb:.2f} s", file=sys.stderr, flush=True)
    if S0 > 0:
        # The extracted directions are long at this configuration (the starts
        # z0 = P g lie far out in the box, and 2000 steps of 0.003 move each
        # coordinate by a few units), so no step along them from these starts
        # stays in the box and lowers f: the whole path's augmentation makes
        # no move.  The same kernel on the same starts with B's columns as D:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        Dcols = torch.tensor(np.ascontiguousarray(B.T).astype(np.int8), device="cuda")
        xa, fa, sa, ba = G.augment(ctx, prob, obj, Dcols, starts)
        torch.cuda.synchronize()
        ela = time.perf_counter() - ta
        out["augment_trajectory_leg"] = {
            "directions": f"the {d} columns of B (and their negations)", "starts": S0,
            "moves": int(sa.sum().item()), "ms": ela * 1e3, "best_f": float(fa[ba].item()),
            "moves_per_s": int(sa.sum().item()) / ela,
            "note": "the whole path's augmentation over the filtered set makes "
                    f"{recs[-1]['mean_steps'] * S0:.0f} moves: its directions are long (in one measured step of "
                    "this configuration the shortest of 26.3 M had l1 norm 4115 and 293 nonzeros), so from these "
                    "starts no step stays in [l, u] and lowers f"}
        del Dcols, xa, fa, sa
    ctx.close()
    del starts
    torch.cuda.empty_cache()
    if args.serve_leg > 0:
        r = _serve_run(args.serve_leg, n_max=300)
        out["serving_leg"] = dict(r, note="short leg of the serving configuration with n capped at 300 (host "
                                          "kernel bases of the iid law take about 2 minutes at n = 1000)")
        print(f"[quartic] serving leg {r['completed_per_s']:.1f} req/s, p99 {r['latency_ms']['p99']:.0f} ms",
              file=sys.stderr, flush=True)
    if cpu is not None:
        cpu["cpu_model"] = _cpu_model()
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def bench_qp(args):
    """The QP workload (m = 20, n = 100, d = 80), 65536 box starts x 2000
    binary32 iterations: extraction, filter and augmentation per step."""
    from paper_2412_13576_amd import workloads as W

    inst = W.qp_instance(2000)
    # the host baseline runs first, before anything here touches the GPU
    cpu = None if args.no_cpu_baseline else _cpu_baseline(inst, args.iters)

    import torch

    from paper_2412_13576_amd import graver as G

    B, P = G.kernel_basis(inst.A)              # host C++ (Lemma 3.1 + LLL), not timed
    n, d = B.shape
    N, T, S0 = args.starts or 65536, args.iters, args.aug_starts
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    obj = G.objective("quadratic", Q=inst.Q, c=inst.c)
    starts_h = W.feasible_walk_starts(inst.x0, B.T.copy(), inst.l, inst.u, S0, seed=7, walk_len=32)
    starts = torch.tensor(starts_h, device="cuda")
    pool_cap = 1 << 23
    keys_buf_cap = pool_cap

    def step(seed):
        prec = G.GRAVER_FP32 if args.precision == "fp32" else G.GRAVER_BF16
        prm = G.extract_params(N, T, precision=prec, init_mode=0, seed=seed, pool_capacity=pool_cap,
                               polish_iters=args.polish if args.precision == "bf16" else 0,
                               any_order=True)  # the filter sorts
        keys, st = G.extract(ctx, prob, prm, keys_cap=keys_buf_cap)
        F = G.filter_minimal(ctx, keys)
        x, f, steps, best = G.augment(ctx, prob, obj, F, starts)
        return keys.shape[0], F.shape[0], st, f, steps, best

    for w in range(args.warmup):
        step(1000 + w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for k in range(args.steps):
        recs.append(step(2000 + k))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el * 1000.0 / args.steps

    n_keys = [r[0] for r in recs]
    n_min = [r[1] for r in recs]
    desc_ms = float(np.mean([r[2]["ms_descent"] for r in recs]))
    roof = descent_roofline(n, d, N, T, desc_ms, bf16_iters=0 if args.precision == "fp32" else T - args.polish)
    out = {
        "metric": "start-iterations/s (whole path: extraction + filter + augmentation)",
        "value": N * T * args.steps / el,
        "unit": "start-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16+f32",
        "data": "synthetic",
        "config": {"workload": "qp_m20_n100: m=20, n=100 (d=80), A in {-1,0,1} density 0.3, "
                               "nonconvex dense quadratic f, box [-10,10]",
                   "starts": N, "iters": T, "aug_starts": S0,
                   "precision": "fp32-mfma" if args.precision == "fp32" else f"bf16-mfma, {args.polish} fp32 polish"},
        "verified_directions_per_s": float(np.mean(n_keys)) / (ms_step * 1e-3),
        "descent_start_iterations_per_s": N * T / (desc_ms * 1e-3),
        "extract": {k: float(np.mean([r[2][k] for r in recs])) for k in
                    ("emit_events", "inbox_events", "unique", "verified", "out_of_range",
                     "ms_init", "ms_descent", "ms_verify", "ms_sort")},
        "filtered": float(np.mean(n_min)),
        "aug_best_f": float(recs[-1][3][recs[-1][5]].item()),
        "aug_mean_steps": float(recs[-1][4].double().mean().item()),
        "roofline": {"bound": "mfma", "kernel": "k_descent_f32", "achieved": roof["achieved"],
                     "peak": roof["peak"], "unit": "TFLOP/s", "frac": roof["frac"],
                     "traffic": _measured_traffic(N, T, args.precision),
                     "algorithmic": "4*n*d flop per start-iteration (B z forward + B^T sign backward)",
                     "peak_note": roof["peak_note"]},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--starts", type=int, default=0, help="starts (default: the configuration's)")
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--aug-starts", type=int, default=200)
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32")
    ap.add_argument("--polish", type=int, default=200, help="bf16: final iterations in binary32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config", choices=["quartic", "qp", "precision", "batch", "serve", "augment"],
                    default="quartic",
                    help="quartic: the whole path on the largest single-GPU configuration (default); qp: the "
                         "QP workload; the others measure the precision, batching and serving configurations")
    ap.add_argument("--serve-leg", type=int, default=60,
                    help="quartic: requests of the short serving leg reported beside (0: none)")
    ap.add_argument("--no-bf16-line", action="store_true", help="quartic: skip the bf16 + polish step")
    ap.add_argument("--no-dense-leg", action="store_true",
                    help="quartic: skip the matrix-core extraction of the same launch")
    ap.add_argument("--requests", type=int, default=300, help="serve: number of requests")
    ap.add_argument("--n-max", type=int, default=1000, help="serve: largest n of the request law")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (a kernel of known traffic, for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the hot path is measured on one MI355X "
              "(multi-GPU sharding is described in DESIGN.md, not run)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        _copy_calibration()
    {"quartic": bench_quartic, "qp": bench_qp, "precision": bench_precision, "batch": bench_batch,
     "serve": bench_serve, "augment": bench_augment}[args.config](args)



if __name__ == "__main__":
    main()
