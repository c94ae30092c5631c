#!/usr/bin/env python3
"""Latent-step benchmark on one MI355X.

Workload (the cake-scale single instance): 200,000 particles in a 0.3 x 0.3 x 0.15 slab,
8,192 of them resampled uniformly each step as integration and sample particles, r = 6,
three width-128 field MLPs (Xavier-uniform weights, seed 0), 128^3 grid, dt = 5e-5, a
knife moving down at 0.5 m/s, 2 Gauss-Newton iterations, and all 200,000 particles
decoded every step. A "step" is one whole latent step: field inference with the latent
Jacobian, P2G, grid update + G2P, two Gauss-Newton iterations, decode.

Prints one JSON line: latent steps/s over exactly --steps graph-replayed steps (inputs
resident in HBM), decoded points/s, p50/p99 per-step device latency, the decode kernel's
MFMA roofline fraction measured with HIP events on its stream, the relative position
error against the FP64 oracle, and the oracle itself timed on the host cores.
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

METRIC = "latent steps/s & decoded pts/s vs plain FP32; p99 step latency at 1e-4 err"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}   # dense MFMA peaks of MI355X


def primal_flops(width: int, r: int, d: int) -> int:
    """Algorithmic FLOP per point of one field MLP: 2 [(3 + r) w + 4 w^2 + w d]."""
    return 2 * ((3 + r) * width + 4 * width * width + width * d)


def tangent_flops(width: int, r: int) -> int:
    """Forward-mode latent Jacobian of g on top of the primal: r (8 w^2 + 6 w)."""
    return r * (8 * width * width + 6 * width)


def step_flops(width, r, n_int, n_samp, n_part, gn_iters=2):
    a = n_int * (2 * primal_flops(width, r, 3) + primal_flops(width, r, 6) + primal_flops(width, r, 9))
    a += n_samp * tangent_flops(width, r)
    g = (gn_iters - 1) * n_samp * (primal_flops(width, r, 3) + tangent_flops(width, r))
    d = n_part * primal_flops(width, r, 3)
    return a + g + d


def cpu_baseline(workload, n_steps: int):
    """The FP64 oracle on this host's cores, on the first n_steps of the same workload."""
    from oracle.step import OracleSim
    try:
        import threadpoolctl
        threads = max(i["num_threads"] for i in threadpoolctl.threadpool_info()) or 1
    except Exception:
        threads = os.cpu_count() or 1
    o = OracleSim(workload)
    t0 = time.perf_counter()
    for _ in range(n_steps):
        o.step(1)
        xdec = o.decode()
    dt = time.perf_counter() - t0
    return o, xdec, {"value": n_steps / dt, "unit": "latent steps/s", "cores": int(threads),
                     "kind": "oracle",
                     "sample": f"first {n_steps} steps of the same workload, each with the "
                               f"200k-particle decode; NumPy float64, BLAS threads={threads}; "
                               f"{dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=("fp32", "bf16"), default="fp32")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the latent step of one "
                                   "simulation is not sharded across GPUs in this build",
                          "n_gpus": args.gpus}))
        return 2

    import torch

    import synth
    from paper_2310_17790_amd import _abi as A
    from paper_2310_17790_amd.sim import Sim

    K, W = args.steps, args.warmup
    width, r, P, NI = 128, 6, 200_000, 8192
    wl = synth.cake_slab(seed=0, r=r, width=width, n=P, n_integration=NI, steps=K + W,
                         plan_steps=min(K + W, 128))
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    sim = Sim(wl, precision=args.precision, stream=stream)
    sim.step(max(W, 1), stream=stream)
    stream.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        evs[i][0].record(stream)
        sim.step(1, stream=stream)
        evs[i][1].record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    status, flags = sim.flags(stream=stream)

    # Dominant kernel: the decode MLP over all 200k particles (the same kernel and launch
    # shape the step uses), timed with HIP events on its stream.
    out = torch.empty(3 * P, dtype=torch.float32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_dec = max(K, 10)
    A.nsf_decode(sim.handle, None, P, out.data_ptr(), stream.cuda_stream)
    e0.record(stream)
    for _ in range(n_dec):
        A.nsf_decode(sim.handle, None, P, out.data_ptr(), stream.cuda_stream)
    e1.record(stream)
    stream.synchronize()
    dec_ms = e0.elapsed_time(e1) / n_dec
    dec_flop = P * primal_flops(width, r, 3)
    achieved = dec_flop / (dec_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]

    # Accuracy at this workload and the CPU baseline: the oracle and a fresh GPU sim run
    # the same first steps; compare decoded positions (the paper's delta, Sec. 6).
    res_cpu, delta_x = None, None
    if not args.no_cpu_baseline:
        oracle, x_ref, res_cpu = cpu_baseline(wl, args.cpu_steps)
        chk = Sim(wl, precision=args.precision, stream=stream)
        chk.step(args.cpu_steps, stream=stream)
        stream.synchronize()
        xg = chk.buffer(A.NSF_BUF_XDEC).reshape(3, -1).double().cpu().numpy().T
        delta_x = float(np.sqrt(((xg - x_ref) ** 2).sum() / (x_ref ** 2).sum()))

    steps_per_s = K / wall
    flop_step = step_flops(width, r, NI, NI, P)
    line = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "latent steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * wall / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (seeded Xavier-uniform fields, uniform slab, per-step uniform resampling)",
        "config": {"workload": "cake-scale single instance: 200,000 particles, 8,192 integration = "
                               "sample particles resampled per step, r=6, width-128 fields, 128^3 "
                               "grid, dt=5e-5, knife, 2 Gauss-Newton iterations, decode all "
                               "particles every step",
                   "particles": P, "integration": NI, "r": r, "width": width, "grid": 128,
                   "precision": args.precision},
        "decoded_pts_per_s": steps_per_s * P,
        "p50_step_ms": float(np.percentile(lat, 50)),
        "p99_step_ms": float(np.percentile(lat, 99)),
        "step_tflops": flop_step / (wall / K) / 1e12,
        "delta_x_vs_oracle": delta_x,
        "delta_x_steps": None if delta_x is None else args.cpu_steps,
        "device_flags": flags,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": f"decode MLP (fields_dense_kernel, width {width}), {P} points, "
                               f"{primal_flops(width, r, 3)} FLOP/point",
                     "avg_ms": dec_ms},
        "cpu_baseline": res_cpu,
    }
    print(json.dumps(line))
    return 0 if status == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
