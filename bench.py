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
PEAK_HBM = 8000.0       # GB/s

# HBM traffic of the descent kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a copy of known
# size.  The summary records a hash of the kernel's sources; a figure taken
# on other sources is not reported.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_descent_f32_qp_m20_n100_hbm_traffic.md")
KERNEL_SOURCES = ["paper_2412_13576_amd/csrc/descent_f32.hip", "paper_2412_13576_amd/csrc/graver_internal.h",
                  "paper_2412_13576_amd/csrc/pool_device.h"]


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _measured_traffic(N, T, precision):
    """Bytes per descent launch recorded for these sources and this launch
    shape, or None."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith(("#", "|", "`")))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_sources_sha256():
        return None
    if kv.get("launch") != f"N={N} T={T} {precision}":
        return None
    return float(kv["hbm_bytes_per_launch"])


def _cpu_baseline(inst, B, P, T, seconds_target=15.0):
    """Oracle (binary64 numpy, one core) on a bounded sample of starts at the
    full T: start-iterations/s."""
    from oracle import philox
    from oracle import surrogate as S

    n_sample = 384
    _, z0 = philox.box_starts(P, inst.l, inst.u, n_sample, seed=99)
    t = time.perf_counter()
    iters = T
    S.extract(inst.A, B, inst.l, inst.u, z0, iters, S.AdamParams(), check_kernel=False)
    el = time.perf_counter() - t
    return {"value": n_sample * iters / el, "unit": "start-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_sample} starts x {iters} iterations of the same instance (binary64 numpy, "
                      f"single thread), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--starts", type=int, default=65536)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--aug-starts", type=int, default=200)
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32")
    ap.add_argument("--polish", type=int, default=200, help="bf16: final iterations in binary32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (a kernel of known traffic, for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the hot path is measured on one MI355X "
              "(multi-GPU sharding is described in DESIGN.md, not run)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_13576_amd import graver as G
    from paper_2412_13576_amd import workloads as W

    inst = W.qp_instance(2000)
    B, P = G.kernel_basis(inst.A)              # host C++ (Lemma 3.1 + LLL), not timed
    n, d = B.shape
    N, T, S0 = args.starts, args.iters, args.aug_starts
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
                               polish_iters=args.polish if args.precision == "bf16" else 0)
        keys, st = G.extract(ctx, prob, prm, keys_cap=keys_buf_cap)
        F = G.filter_minimal(ctx, keys)
        x, f, steps, best = G.augment(ctx, prob, obj, F, starts)
        return keys.shape[0], F.shape[0], st, f, steps, best

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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
    flops = 4.0 * n * d * N * T
    achieved = flops / (desc_ms * 1e-3) / 1e12
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
        "roofline": {"bound": "mfma", "kernel": "k_descent_f32", "achieved": achieved,
                     "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": _measured_traffic(N, T, args.precision),
                     "algorithmic": "4*n*d flop per start-iteration (B z forward + B^T sign backward)"},
    }
    if not args.no_cpu_baseline:
        from oracle import lattice
        Bo = lattice.kernel_basis(inst.A)
        Po = lattice.coordinate_projector(Bo) if n <= 100 else P
        out["cpu_baseline"] = _cpu_baseline(inst, Bo, Po, T)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
