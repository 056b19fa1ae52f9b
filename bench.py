#!/usr/bin/env python
"""Benchmark: auxiliary-Kalman MCMC steps/s on one MI355X.

Workload: the d_x = 64, T = 4096 latent field on a periodic grid (nearest-
neighbour F, squared-exponential Q + 1e-6 jitter) observed through Student-t
noise (nu = 3, scale 0.5) at 32 evenly spaced sites; second-order proposal,
fixed step size delta; one chain.  Synthetic data and normals, all seeded.

One "step" is one full auxiliary-Kalman MH step: aux draw + linearisation,
parallel filter (block fold, tree, block re-scan), pathwise sampler (element
build, fold, tree, final), reverse linearisation + filter, MH reduction and
select.  Inputs (model, data, normals, uniforms) are resident in HBM before
the timed region starts.

Prints ONE JSON line (rank 0).  With --gpus > 1 it exits with a message: this
build measures a single GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "aux-Kalman MCMC steps/s at d_x=64,T=4096; batched+adjoint vs plain, same GPU"
PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0


def fold_flops_per_step(d: int, first: bool, t0: bool) -> float:
    """Algorithmic flops of one block-fold step at dimension d (2 per multiply-
    add, triangular and symmetric products counted at their reduced cost):
    predict F C F' (2 GEMMs), Cholesky + triangular inverse of S, X = L^{-1} P^p,
    X'X, and for blocks past the first F A, Y = L^{-1} F A, Y'Y, X'Y."""
    d3 = float(d) ** 3
    f = (0.0 if t0 else 4.0 * d3) + (2.0 / 3.0) * d3 + 2.0 * d3
    if not first:
        f += 2.0 * d3 + d3 + d3 + 2.0 * d3
    return f


def fold_flops_per_launch(N: int, d: int, B: int) -> float:
    tot = 0.0
    for t in range(N):
        tot += fold_flops_per_step(d, first=(t < B), t0=(t == 0))
    return tot


def auto_block(N: int, d: int) -> int:
    D = 16 if d <= 16 else (32 if d <= 32 else 64)
    teams = 1 if D == 64 else (4 if D == 32 else 8)
    target = 256 * teams
    B = max(4, (N + target - 1) // target)
    return min(B, N)


def cpu_baseline(w, n_steps: int) -> dict:
    """The FP64 oracle (sequential C, one thread) on a bounded sample: n_steps
    full MH steps of the same workload, from the same state and normals."""
    import numpy as np
    import oracle
    M = oracle.Model(**w.oracle_kwargs())
    xi = w.normals(n_steps)
    un = w.uniforms(n_steps)
    x = w.x_true.copy()
    t0 = time.perf_counter()
    for k in range(n_steps):
        r = oracle.mh_step(M, w.y, x, w.delta, w.order, xi[k, 0], xi[k, 1], un[k])
        x = r["x_out"]
    dt = time.perf_counter() - t0
    return {"value": n_steps / dt, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_steps} full MH steps of the same workload (d_x=64, T=4096) by the "
                      f"sequential FP64 C oracle on one host thread, {dt:.1f} s",
            "seconds": dt}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--block", type=int, default=0, help="scan block size (0 = automatic)")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-kernel", default="filter_fold")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "the sampler runs one chain per GPU and no multi-GPU path is built.",
              file=sys.stderr)
        return 2

    import torch
    from paper_2303_00301_amd import workloads as W
    from paper_2303_00301_amd import sampler as S
    from paper_2303_00301_amd import _lib

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = W.latent_field()
    N, d = w.N, w.dx
    B = args.block or auto_block(N, d)
    M = S.DeviceModel.from_workload(w, device=dev)
    y = torch.as_tensor(w.y, dtype=torch.float64, device=dev)
    x = torch.as_tensor(w.x_true, dtype=torch.float64, device=dev).contiguous()
    K, Wm = args.steps, args.warmup
    gen = torch.Generator(device=dev)
    gen.manual_seed(103)
    xi = torch.randn((K + Wm, 2, N, d), dtype=torch.float64, device=dev, generator=gen)
    un = torch.rand((K + Wm,), dtype=torch.float64, device=dev, generator=gen).clamp_(min=1e-300)
    ws = S.Workspace(dev)

    # warm-up
    if Wm:
        S.mh_run(M, y, x, w.delta, w.order, xi[:Wm], un[:Wm], block=B, ws=ws)
    torch.cuda.synchronize()

    lib = _lib.load()
    fam = _lib.FAMILIES[args.roofline_kernel]
    _lib.check(lib.akf_timing_enable(fam, 8 * K + 16), "akf_timing_enable")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    out = S.mh_run(M, y, x, w.delta, w.order, xi[Wm:], un[Wm:], block=B, ws=ws)
    ev1.record()
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    import ctypes as C
    n_l = C.c_int32()
    k_ms = C.c_double()
    _lib.check(lib.akf_timing_collect(C.byref(n_l), C.byref(k_ms)), "akf_timing_collect")
    lib.akf_timing_enable(-1, 0)

    acc = out["accepted"].float().mean().item()
    status_bad = int((out["status"] != 0).sum().item())
    ms_step = ms_total / K
    steps_s = 1000.0 / ms_step

    roof = None
    if n_l.value > 0:
        avg_ms = k_ms.value / n_l.value
        if args.roofline_kernel == "filter_fold":
            flops = fold_flops_per_launch(N, d, B)
        else:
            flops = float("nan")
        achieved = flops / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                "kernel": f"k_filter_fold<64> ({args.roofline_kernel})",
                "avg_launch_ms": avg_ms, "launches": n_l.value,
                "flops_per_launch": flops}

    res = {
        "metric": METRIC,
        "value": steps_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"latent_field_d{d}_T{N}: periodic-grid Gaussian dynamics, "
                               f"Student-t(3, 0.5) at 32 sites, order-2 proposal, one chain",
                   "d_x": d, "T": N, "chains": 1, "order": w.order, "delta": w.delta,
                   "scan_block": B},
        "time_steps_per_s": steps_s * N,
        "acceptance": acc,
        "rejected_by_status": status_bad,
        "roofline": roof,
    }
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
