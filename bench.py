#!/usr/bin/env python3
"""Throughput of the fused D3Q19 BGK + dynamic-IB time step on one MI355X.

Workload: the prolate capsule in shear, 128x64x128 lattice (1 048 576 nodes), tau drawn from
seed 0, walls at shear rate 1e-4, prolate spheroid a=12, b=c=6, level-4 mesh (2562 vertices,
5120 markers), Ca=0.05, k_b = 0.01 k_s0, FP32 shifted populations.  One step = MLS forcing and
spreading, the fused collide+stream sweep, window moments, probe stresses and the membrane
update (all HIP kernels of the library).  value = lattice node updates per second (MLUPS) over
the timed steps.  The sweep's average launch duration comes from start/end events stamped by
every sweep launch's own dispatch packet on the lattice's stream inside the timed region.
`--workload prolate256` runs the same physics at 256x128x256 (level-5 mesh), a working set
larger than the Infinity Cache; `--workload settling384` the 96x96x384 closed box with a rigid
settling sphere in FP16 shifted storage (working set 269 MB).  `--mode batch` and `--mode serve` run the batched and served
forms (64 capsule jobs; a Poisson stream of capsule and settling jobs).

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

# HBM bytes per launch of the FP32 sweep on the 128x64x128 case, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters scaled by a plain copy of known size (fetch x2.0, write x1.0).  Reported
# only while the sweep's sources hash to the value they had when the counters were taken.
# every 10th sweep launch of the timed region carries start/end events (evenly spread; the
# events' own cost stays out of the other steps)
TIMING_PERIOD = 10
SWEEP_SOURCES = ("paper_2207_06029_amd/csrc/lbib_lattice.hip", "paper_2207_06029_amd/csrc/lbib_internal.h")
SWEEP_TRAFFIC = {
    # FETCH_SIZE 39,272.2 KiB x 2.0 + WRITE_SIZE 77,824.0 KiB x 1.0 per dispatch
    "prolate128": {"sha256": "ee6bce77e602b0664cba62131773ab5519d11e4d65284433acfc148a62bd137e",
                   "bytes": 160121242},
    # FETCH_SIZE 313,582.6 KiB x 2.0 + WRITE_SIZE 622,592.0 KiB x 1.0 per dispatch
    "prolate256": {"sha256": "ee6bce77e602b0664cba62131773ab5519d11e4d65284433acfc148a62bd137e",
                   "bytes": 1279751373},
    # FETCH_SIZE 89,838.1 KiB x 2.0 + WRITE_SIZE 131,328.0 KiB x 1.0 per dispatch (the FP16
    # reads are 1.36x their algorithmic bytes, probably since 192 B rows misalign the y-shifted streams)
    "settling384": {"sha256": "ee6bce77e602b0664cba62131773ab5519d11e4d65284433acfc148a62bd137e",
                    "bytes": 318468301},
}


def sources_sha256(paths=SWEEP_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    rec = SWEEP_TRAFFIC.get(workload, {})
    if rec.get("sha256") and rec["sha256"] == sources_sha256():
        return rec["bytes"]
    return None


# Plain FP32 workloads: the prolate capsule in shear at 128x64x128 (the headline case) and the
# same physics at twice the linear size, whose populations (2 x 637 MB) do not fit the 256 MB
# Infinity Cache.
# name -> (generator in inputs, its arguments after the seed (None: seeded), description)
WORKLOADS = {
    "prolate128": ("prolate_shear", None, "prolate capsule in shear, level-4 mesh (2562 vertices, 5120 markers)"),
    "prolate256": ("prolate_shear_large", None, "prolate capsule in shear, level-5 mesh (10242 vertices, 20480 markers)"),
    "settling384": ("settling_sphere", (1.5, 1), "rigid sphere settling in a closed box, density ratio 1.5, "
                                                 "level-4 mesh (2562 vertices, 5120 markers)"),
}


def cpu_baseline(job, target_s: float = 15.0) -> dict:
    """The FP64 oracle (as it stands) on the same workload, timed on the host's cores."""
    import oracle
    cores = max(1, min(16, os.cpu_count() or 1))
    oracle.set_threads(cores)
    lat = oracle.Lattice(job.lattice)
    lat.add_body(job.body, job.xyz, job.tri)
    lat.step(1)   # thread start-up and first touch, untimed
    t0 = time.perf_counter()
    lat.step(2)
    one = (time.perf_counter() - t0) / 2.0
    n = max(1, min(5000, int(target_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    lat.step(n)
    dt = time.perf_counter() - t0
    mlups = job.lattice.n * n / dt / 1e6
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{n} full steps (IB + collide/stream + membrane) of the same "
                      f"{job.lattice.nx}x{job.lattice.ny}x{job.lattice.nz} case after 3 steps, "
                      f"{dt:.1f} s, FP64, OpenMP over lattice nodes"}


def calibrate_copy(nbytes: int, reps: int) -> None:
    """Plain device copies of known size: the reference for scaling the HBM byte counters, and
    the read+write bandwidth a streaming kernel can reach (timed with HIP events)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    us = t0.elapsed_time(t1) * 1e3 / reps
    print(json.dumps({"calibration_copy_bytes": nbytes, "reps": reps, "avg_us": round(us, 3),
                      "read_plus_write_GBs": round(2 * nbytes / us / 1e3, 1)}))


def bench_batch(args) -> dict:
    """64 capsule-in-shear jobs in shared launches (FP16 shifted storage, hipGraph, autotuned
    sweep shape) against the plain form: the same jobs one at a time with FP32 storage."""
    import torch
    from paper_2207_06029_amd import api
    from paper_2207_06029_amd import inputs as I
    jobs = I.capsule_batch(seed=0, njobs=64, storage=I.STORE_F16, steps=2000)
    nodes = sum(j.lattice.n for j in jobs)
    stream = torch.cuda.current_stream()
    bt = api.Batch(jobs, storage=I.STORE_F16, autotune=True, use_graph=True, stream=stream)
    bt.step(args.warmup)
    bt.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bt.sync()
    per_step = wall / args.steps
    # sweep-only timing of the batched launch (events around the sweep, no graph)
    lat0 = bt.lattice(0)
    lat0.set_timing(True)
    bt.step(50)
    sweep_ms, nsweep = lat0.kernel_time(0)
    lat0.set_timing(False)
    sweep_s = sweep_ms / nsweep / 1e3
    bytes_sweep = 2 * 19 * 2 * nodes
    # plain per-job form
    plain_s = 0.0
    k = max(10, args.steps // 10)
    for idx, j in enumerate([] if args.skip_plain else jobs):
        if idx % 16 == 0:
            print(f"[batch] plain per-job form: job {idx}/{len(jobs)}", file=sys.stderr, flush=True)
        lat = api.Lattice(j.lattice.__class__(**{**j.lattice.__dict__, "storage": I.STORE_F32}), stream=stream)
        lat.add_body(j.body, j.xyz, j.tri)
        lat.step(5)
        lat.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(k)
        torch.cuda.synchronize()
        plain_s += (time.perf_counter() - t0) / k
        lat.sync()
        lat.destroy()
    steps_job = jobs[0].steps
    return {
        "metric": METRIC, "mode": "batch",
        "value": round(nodes / per_step / 1e6, 2), "unit": "MLUPS",
        "jobs_per_hour": round(3600.0 / (per_step * steps_job) * len(jobs), 1),
        "plain_jobs_per_hour": round(3600.0 / (plain_s * steps_job) * len(jobs), 1) if plain_s else None,
        "plain_mlups": round(nodes / plain_s / 1e6, 2) if plain_s else None,
        "ms_per_batched_step": round(per_step * 1e3, 4),
        "launch_shape": list(bt.launch_shape()),
        "roofline": {"bound": "hbm", "achieved": round(bytes_sweep / sweep_s / 1e9, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(bytes_sweep / sweep_s / 1e9 / PEAK_HBM_GBS, 4),
                     "kernel": "k_sweep<half,collide> (64 jobs)", "bytes_per_launch": bytes_sweep,
                     "avg_launch_us": round(sweep_s * 1e6, 3)},
        "config": {"workload": "64 capsule-in-shear jobs, cubic edges from {32..96}, spheres and "
                               "oblate capsules, level 3/4 meshes, FP16 shifted storage",
                   "nodes_total": nodes, "steps_timed": args.steps},
        "dtype": "f16-storage/f32-compute", "data": "synthetic", "n_gpus": 1,
    }


def bench_serve(args) -> dict:
    """Poisson arrivals (mean 4 jobs/s) of capsule-shear and settling jobs served with
    continuous batching and a device-memory budget; time-to-result percentiles and throughput,
    then the same stream through a one-job-at-a-time FIFO of the plain FP32 form."""
    import numpy as np
    import torch
    from paper_2207_06029_amd import api
    from paper_2207_06029_amd import inputs as I

    def run(stream_jobs, slots, storage, budget, tick):
        srv = api.Server(hbm_budget_bytes=budget, max_slots=slots, steps_per_tick=tick,
                         storage=storage, stream=torch.cuda.current_stream())
        pending = sorted(stream_jobs, key=lambda j: j.arrival_s)
        t_start = time.perf_counter()
        done, nodes_steps = [], 0.0
        i = 0
        last_note = 0.0
        while len(done) < len(pending):
            now = time.perf_counter() - t_start
            if now - last_note > 10.0:
                st = srv.stats()
                print(f"[serve slots={slots}] t={now:.0f}s submitted={i} done={len(done)} "
                      f"resident={st['resident']} queued={st['queued']}", file=sys.stderr, flush=True)
                last_note = now
            while i < len(pending) and pending[i].arrival_s <= now:
                srv.submit(pending[i])
                i += 1
            srv.tick()
            for r in srv.poll():
                done.append(r)
            if i < len(pending) and srv.stats()["resident"] == 0 and srv.stats()["queued"] == 0:
                time.sleep(max(0.0, pending[i].arrival_s - (time.perf_counter() - t_start)))
            if time.perf_counter() - t_start > args.serve_window * 6 + 120:
                break
        wall = time.perf_counter() - t_start
        st = srv.stats()
        lat = np.array([(r["t_finish_ns"] - r["t_submit_ns"]) * 1e-9 for r in done])
        ok = sum(1 for r in done if r["status"] == 0)
        by_tag = {j.tag: j for j in pending}
        failures = []
        for r in done:
            if r["status"] != 0:
                j = by_tag[r["tag"]]
                failures.append({"status": r["status"], "kind": j.kind, "dims": [j.lattice.nx, j.lattice.ny, j.lattice.nz],
                                 "nv": int(len(j.xyz)), "mass_ratio": round(j.body.mass_ratio, 3),
                                 "ks0": round(j.body.ks0, 5), "kb": round(j.body.kb, 6),
                                 "tau": round(j.lattice.tau, 3), "steps_done": r["steps_done"]})
        return {"jobs": len(done), "ok": ok, "failures": failures[:40], "wall_s": round(wall, 2),
                "jobs_per_hour": round(len(done) / wall * 3600, 1),
                "mlups": round(st["node_updates"] / wall / 1e6, 1),
                "p50_s": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
                "p99_s": round(float(np.percentile(lat, 99)), 3) if len(lat) else None}

    jobs = I.serving_stream(seed=0, rate_per_s=4.0, window_s=args.serve_window,
                            storage=I.STORE_F16)
    served = run(jobs, slots=64, storage=I.STORE_F16, budget=32 << 30, tick=100)
    plain = run(I.serving_stream(seed=0, rate_per_s=4.0, window_s=args.serve_window,
                                 storage=I.STORE_F32), slots=1, storage=I.STORE_F32,
                budget=32 << 30, tick=100)
    return {"metric": METRIC, "mode": "serve", "value": served["jobs_per_hour"], "unit": "jobs/h",
            "served": served, "plain_fifo": plain,
            "config": {"workload": f"Poisson arrivals 4 jobs/s over {args.serve_window:.0f} s: "
                                   "capsule-shear and settling jobs, lattices 48^3..128x64x128, "
                                   "meshes 642-10242 vertices, 2000-10000 steps, FP16 storage, "
                                   "32 GiB budget, 64 slots, 100 steps per tick"},
            "dtype": "f16-storage/f32-compute", "data": "synthetic", "n_gpus": 1}


def make_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", type=int, default=0, help="bytes: run only a copy of that size")
    ap.add_argument("--graph", action="store_true",
                    help="also time the same steps replayed from a captured hipGraph")
    ap.add_argument("--mode", choices=["plain", "batch", "serve"], default="plain")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="prolate128",
                    help="plain mode: prolate capsule in shear at 128x64x128 (default) or 256x128x256, "
                         "or the FP16 rigid sphere settling in a 96x96x384 box")
    ap.add_argument("--serve-window", type=float, default=60.0)
    ap.add_argument("--skip-plain", action="store_true",
                    help="batch mode: time only the batched form (no per-job comparison)")
    ap.add_argument("--sources-sha256", action="store_true",
                    help="print the hash of the sweep's sources and exit")
    return ap


def main() -> int:
    args = make_parser().parse_args()
    if args.sources_sha256:
        print(sources_sha256())
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        return 2
    if args.calib_copy:
        calibrate_copy(args.calib_copy, 10)
        return 0
    if args.mode == "batch":
        print(json.dumps(bench_batch(args)))
        return 0
    if args.mode == "serve":
        print(json.dumps(bench_serve(args)))
        return 0

    import torch
    from paper_2207_06029_amd import api
    from paper_2207_06029_amd import inputs as I

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    gen, gen_args, wl_text = WORKLOADS[args.workload]
    job = getattr(I, gen)(*gen_args) if gen_args is not None else getattr(I, gen)(args.seed)
    spec = job.lattice
    s_bytes = 4 if spec.storage == I.STORE_F32 else 2
    lat = api.Lattice(spec, stream=stream)
    b = lat.add_body(job.body, job.xyz, job.tri)
    lat.step(args.warmup)
    lat.sync()

    lat.set_timing(TIMING_PERIOD)
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
    bytes_per_launch = 2 * 19 * s_bytes * n  # algorithmic: read and write 19 stored values per node
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
        "dtype": "f32" if s_bytes == 4 else "f16-storage/f32-compute",
        "data": "synthetic",
        "config": {"workload": f"{wl_text}, {spec.nx}x{spec.ny}x{spec.nz} D3Q19, tau={spec.tau:.4f}"
                               + (f" (seed {args.seed})" if gen_args is None else "")
                               + (", FP32 shifted populations" if s_bytes == 4 else ", FP16 shifted populations"),
                   "lattice": [spec.nx, spec.ny, spec.nz], "markers": int(len(job.tri)), "name": args.workload,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(args.workload),
                     "kernel": "k_sweep<float,collide>" if s_bytes == 4 else "k_sweep<half,collide>",
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": round(sweep_avg_s * 1e6, 3)},
        "breakdown": {"sweep_us_avg": round(sweep_avg_s * 1e6, 3),
                      "sweep_launches_timed": nsweep,
                      "step_us_avg_events": round(step_ms / max(nstep, 1) * 1e3, 3),
                      "sweep_share_of_step": round(sweep_avg_s * 1e3 * nstep / max(step_ms, 1e-9), 4),
                      "sweep_only_mlups": round(n / sweep_avg_s / 1e6, 1)},
    }
    if args.graph:
        # same job as a one-job batch whose steps replay a captured two-step hipGraph
        bt = api.Batch([job], storage=spec.storage, use_graph=True, stream=stream)
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
