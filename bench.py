"""Benchmark: velocity-node updates per second of the IMEX-SSP3(4,3,3) MP-9
lattice Boltzmann step on one MI355X, FP64 and FP32 storage.

Workload: 2D four-quadrant Riemann problem on 4096 x 4096 cells over [0,1]^2,
8 x 8 Gauss-Hermite velocities per distribution (phi and chi: 128 planes per
cell), K = 2 (gamma = 7/5), tau = 1e-7, dt = 0.5 dx / max|p| (CFL 0.5),
outflow walls; seeded quadrant states (synthetic, see workloads.py).

One step = the three fused stage passes over all 2^31 populations.  The
JSON line reports the FP64 throughput as ``value`` (the plain FP64 method),
the FP32-storage run beside it, per-pass HIP-event timings, the roofline of
the dominant pass, and the FP64 CPU oracle timed on a bounded patch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PMAX8 = 4.144547186125894  # largest root of He_8
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E spec peak
METRIC = "velocity-node updates/s per IMEX step, FP32 vs FP64, % of HBM roofline"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_bytes(planes, cells, elem, nf):
    """Algorithmic HBM bytes of the three passes (plane-sets read/written,
    FP64 moment sets read/written); see the design notes."""
    ps = planes * cells * elem
    ms = nf * cells * 8
    return {"stage3": 2 * ps + 2 * ms, "stage4": 4 * ps + 3 * ms, "stage5": 3 * ps + 2 * ms}


def run_precision(I, W, N, storage, steps, warmup, seed):
    import torch

    dt = 0.5 / N / PMAX8
    cfg = I.Config(d=2, nx=N, ny=N, q_phi=8, q_chi=8, K=2, tau=1e-7, dt=dt, storage=storage)
    states, k = W.quadrant_states(seed)
    fields = W.riemann_2d(N, N, states)
    s = I.Solver(cfg)
    s.set_equilibrium(*fields)
    if warmup:
        s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = s.step_timed(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ok = s.check_state()
    cells = N * N
    planes = cfg.planes
    vn = cells * planes * steps / wall
    elem = 4 if storage == I.F32 else 8
    pb = pass_bytes(planes, cells, elem, 4)
    per = {k2: ms[i] / steps for i, k2 in enumerate(("stage3", "stage4", "stage5"))}
    step_bytes = sum(pb.values())
    res = {
        "value": vn,
        "ms_per_step": 1e3 * wall / steps,
        "pass_ms": per,
        "pass_bytes": pb,
        "bytes_per_vn_step": step_bytes / (cells * planes),
        "step_gbs": step_bytes / (wall / steps) / 1e9,
        "state_ok": ok == I.OK,
        "seed_offset": k,
    }
    gbs4 = pb["stage4"] / (per["stage4"] * 1e-3) / 1e9
    res["roofline"] = {"bound": "hbm", "kernel": "stage4 (stage2d_kernel<%s, 4>)" %
                       ("float" if elem == 4 else "double"),
                       "achieved": gbs4, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": gbs4 / HBM_PEAK_GBS, "traffic": None}
    del s
    torch.cuda.empty_cache()
    return res, cfg, fields


def cpu_baseline(O, W, cfg, fields, side, steps):
    """The FP64 oracle on a side x side patch of the same workload (centre)."""
    N = cfg.nx
    c0 = N // 2 - side // 2
    sl = (slice(c0, c0 + side), slice(c0, c0 + side))
    pc = O.Config(d=2, nx=side, ny=side, lx=side / N, ly=side / N, q_phi=8, q_chi=8, K=2,
                  tau=cfg.tau, dt=cfg.dt)
    n, ux, uy, T = fields
    F = O.equilibrium(pc, n[sl], ux[sl], uy[sl], T[sl])
    t0 = time.perf_counter()
    O.step(pc, F, steps)
    dt = time.perf_counter() - t0
    vn = side * side * pc.planes * steps / dt
    return {"value": vn, "unit": "VN/s", "cores": 1, "kind": "oracle",
            "sample": f"{side}x{side} cells x 128 planes at the quadrant corner, {steps} "
                      f"IMEX step(s), single-threaded C (-O2), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-side", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=2)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; multi-GPU figures are not "
              "part of it (the sharding design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1909_08390_amd import imexlb as I
    from paper_1909_08390_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log(f"bench: {args.size}^2 cells x 128 planes, FP64, {args.warmup} warmup + {args.steps} steps")
    r64, cfg, fields = run_precision(I, W, args.size, I.F64, args.steps, args.warmup, args.seed)
    log(f"bench: FP64 {r64['value']:.3e} VN/s, {r64['ms_per_step']:.2f} ms/step, passes {r64['pass_ms']}")
    r32 = None
    if not args.no_fp32:
        log("bench: FP32 storage run")
        r32, _, _ = run_precision(I, W, args.size, I.F32, args.steps, args.warmup, args.seed)
        log(f"bench: FP32 {r32['value']:.3e} VN/s, {r32['ms_per_step']:.2f} ms/step, passes {r32['pass_ms']}")
    cpu = None
    if not args.no_cpu:
        import oracle as O
        log("bench: CPU oracle baseline")
        cpu = cpu_baseline(O, W, cfg, fields, args.cpu_side, args.cpu_steps)
        log(f"bench: oracle {cpu['value']:.3e} VN/s")

    out = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "VN/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D four-quadrant Riemann problem, {args.size}x{args.size} cells, "
                        "8x8 Gauss-Hermite velocities per f and g (128 planes), K=2 "
                        "(gamma 7/5), tau=1e-7, CFL 0.5, outflow",
            "cells": args.size * args.size, "planes": 128, "dt": cfg.dt,
            "seed": args.seed + r64["seed_offset"],
        },
        "roofline": r64["roofline"],
        "pass_ms": r64["pass_ms"],
        "bytes_per_vn_step": r64["bytes_per_vn_step"],
        "step_hbm_frac": r64["step_gbs"] / HBM_PEAK_GBS,
        "cpu_baseline": cpu,
    }
    if r32 is not None:
        out["fp32"] = {
            "value": r32["value"], "unit": "VN/s", "dtype": "f32 storage, f64 moments",
            "ms_per_step": r32["ms_per_step"], "pass_ms": r32["pass_ms"],
            "speedup_vs_fp64": r32["value"] / r64["value"],
            "bytes_per_vn_step": r32["bytes_per_vn_step"],
            "step_hbm_frac": r32["step_gbs"] / HBM_PEAK_GBS,
            "roofline": r32["roofline"],
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
