#!/usr/bin/env python3
"""Throughput of the fused D3Q19 BGK + dynamic-IB time step on one MI355X.

Workload: the prolate capsule in shear, 128x64x128 lattice (1 048 576 nodes), tau drawn from
seed 0, walls at shear rate 1e-4, prolate spheroid a=12, b=c=6, level-4 mesh (2562 vertices,
5120 markers), Ca=0.05, k_b = 0.01 k_s0, FP32 shifted populations.  One step = MLS forcing and
spreading, the fused collide+stream sweep, window moments, probe stresses and the membrane
update (all HIP kernels of the library).  value = lattice node updates per second (MLUPS) over
the timed steps.  The sweep's average launch duration comes from HIP events recorded around
every sweep launch on the lattice's stream inside the timed region.

Prints one JSON line.  `--gpus N` with N > 1 exits: this build runs on one GPU.
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

METRIC = "fused D3Q19+IB MLUPS & HBM-roofline %; batched jobs/h, p50/p99 latency"
PEAK_HBM_GBS = 8000.0


def cpu_baseline(job, target_s: float = 15.0) -> dict:
    """The FP64 oracle (as it stands) on the same workload, timed on the host's cores."""
    import oracle
    cores = max(1, min(16, os.cpu_count() or 1))
    oracle.set_threads(cores)
    lat = oracle.Lattice(job.lattice)
    lat.add_body(job.body, job.xyz, job.tri)
    t0 = time.perf_counter()
    lat.step(1)
    one = time.perf_counter() - t0
    n = max(1, min(200, int(target_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    lat.step(n)
    dt = time.perf_counter() - t0
    mlups = job.lattice.n * n / dt / 1e6
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{n} full steps (IB + collide/stream + membrane) of the same "
                      f"{job.lattice.nx}x{job.lattice.ny}x{job.lattice.nz} case after 1 step, "
                      f"{dt:.1f} s, FP64, OpenMP over lattice nodes"}


def calibrate_copy(nbytes: int, reps: int) -> None:
    """Plain device copies of known size, for scaling the HBM byte counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": nbytes, "reps": reps}))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", type=int, default=0, help="bytes: run only a copy of that size")
    ap.add_argument("--graph", action="store_true",
                    help="also time the same steps replayed from a captured hipGraph")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not part of this build", file=sys.stderr)
        return 2
    if args.calib_copy:
        calibrate_copy(args.calib_copy, 10)
        return 0

    import torch
    from paper_2207_06029_amd import api
    from paper_2207_06029_amd import inputs as I

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    job = I.prolate_shear(args.seed)
    spec = job.lattice
    lat = api.Lattice(spec, stream=stream)
    b = lat.add_body(job.body, job.xyz, job.tri)
    lat.step(args.warmup)
    lat.sync()

    lat.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat.sync()  # raises on instability / domain errors
    sweep_ms, nsweep = lat.kernel_time(0)
    step_ms, nstep = lat.kernel_time(1)
    lat.set_timing(False)

    n = spec.n
    mlups = n * args.steps / wall / 1e6
    sweep_avg_s = sweep_ms / nsweep / 1e3
    bytes_per_launch = 2 * 19 * 4 * n      # algorithmic: read and write 19 FP32 per node
    achieved = bytes_per_launch / sweep_avg_s / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"prolate capsule in shear, {spec.nx}x{spec.ny}x{spec.nz} D3Q19, "
                               f"level-4 mesh (2562 vertices, 5120 markers), tau={spec.tau:.4f} "
                               f"(seed {args.seed}), FP32 shifted populations",
                   "lattice": [spec.nx, spec.ny, spec.nz], "markers": int(len(job.tri)),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "kernel": "k_sweep<float,collide>",
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": round(sweep_avg_s * 1e6, 3)},
        "breakdown": {"sweep_us_avg": round(sweep_avg_s * 1e6, 3),
                      "step_us_avg_events": round(step_ms / max(nstep, 1) * 1e3, 3),
                      "sweep_share_of_step": round(sweep_ms / max(step_ms, 1e-9), 4),
                      "sweep_only_mlups": round(n / sweep_avg_s / 1e6, 1)},
    }
    if args.graph:
        # same job as a one-job batch whose steps replay a captured two-step hipGraph
        bt = api.Batch([job], storage=I.STORE_F32, use_graph=True, stream=stream)
        bt.step(args.warmup)
        bt.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.step(args.steps)
        torch.cuda.synchronize()
        gw = time.perf_counter() - t0
        bt.sync()
        out["breakdown"]["graph_ms_per_step"] = round(gw / args.steps * 1e3, 5)
        out["breakdown"]["graph_mlups"] = round(n * args.steps / gw / 1e6, 2)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(job)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
