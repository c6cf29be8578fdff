#!/usr/bin/env python3
"""Throughput of the fused D3Q19 BGK + dynamic-IB time step on one MI355X.

Workload: the prolate capsule in shear, 128x64x128 lattice (1 048 576 nodes), tau drawn from
seed 0, walls at shear rate 1e-4, prolate spheroid a=12, b=c=6, level-4 mesh (2562 vertices,
5120 markers), Ca=0.05, k_b = 0.01 k_s0, FP32 shifted populations.  One step = MLS forcing and
spreading, the fused collide+stream sweep, window moments, probe stresses and the membrane
update (all HIP kernels of the library).  value = lattice node updates per second (MLUPS) over
the timed steps.  The sweep's average launch duration comes from start/end events stamped by
every sweep launch's own dispatch packet on the lattice's stream inside the timed region.
The headline case's populations (2 x 79.7 MB) fit the 256 MB Infinity Cache, so the same run
also reports, under "extra", each with its own sweep fraction of the HBM roofline and its
full-step fraction of roofline MLUPS: the same physics at 256x128x256 (level-5 mesh, 1.27 GB of
populations), the 96x96x384 closed box with a rigid settling sphere in FP16 shifted storage
(269 MB), and the 64-job FP16 batch against the same jobs one at a time in FP32 (jobs/h).
`cpu_baseline` times the FP64 oracle on the host's cores and on one thread (headline case,
32^3 capsule and settling box), with the CPU model and core count.

`--workload prolate256 | settling384` makes one of the extra cases the headline; `--mode batch`
and `--mode serve` run the batched and served forms alone (64 capsule jobs; a Poisson stream of
capsule and settling jobs).

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
INFINITY_CACHE_BYTES = 256 << 20
# the extra workloads of a default run take at least this many timed / warm-up steps
EXTRA_MIN_STEPS = 200
EXTRA_MIN_WARMUP = 20

# every 10th sweep launch of the timed region carries start/end events (evenly spread; the
# events' own cost stays out of the other steps)
TIMING_PERIOD = 10
# HBM bytes per launch of the sweep of each workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# counters scaled by a plain copy of known size (fetch x2.0, write x1.0).  Reported only while the
# sweep's sources hash to the value they had when the counters were taken.
SWEEP_SOURCES = ("paper_2207_06029_amd/csrc/lbib_lattice.hip", "paper_2207_06029_amd/csrc/lbib_internal.h")
SWEEP_TRAFFIC = {
    # FETCH_SIZE 39,290.0 KiB x 2.0 + WRITE_SIZE 77,824.0 KiB x 1.0 per dispatch
    "prolate128": {"sha256": "63188311b0f813a2e409e059f10e986d549799bac5d63470cb94ac1107f12a54",
                   "bytes": 160157653},
    # FETCH_SIZE 314,602.8 KiB x 2.0 + WRITE_SIZE 622,592.0 KiB x 1.0 per dispatch
    "prolate256": {"sha256": "63188311b0f813a2e409e059f10e986d549799bac5d63470cb94ac1107f12a54",
                   "bytes": 1281840677},
    # FETCH_SIZE 90,246.3 KiB x 2.0 + WRITE_SIZE 131,328.0 KiB x 1.0 per dispatch: the FP16 reads
    # are 1.37x their algorithmic bytes, all in 128 B requests (the shifted reads of 192 B rows
    # fetch lines that the neighbouring tiles fetch again)
    "settling384": {"sha256": "63188311b0f813a2e409e059f10e986d549799bac5d63470cb94ac1107f12a54",
                    "bytes": 319304238},
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


def host_info() -> dict:
    """CPU model and the cores this process may run on (the GPU machine's share may be smaller
    than what the kernel reports)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": nproc, "os_cpu_count": os.cpu_count()}


def oracle_mlups(job, threads: int, target_s: float) -> dict:
    """The FP64 oracle (as it stands) stepping job on `threads` host threads for about
    target_s seconds after one untimed step (thread start-up, first touch)."""
    import oracle
    oracle.set_threads(threads)
    lat = oracle.Lattice(job.lattice)
    if job.body is not None:
        lat.add_body(job.body, job.xyz, job.tri)
    lat.step(1)
    t0 = time.perf_counter()
    lat.step(1)
    one = time.perf_counter() - t0
    n = max(1, min(5000, int(target_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    lat.step(n)
    dt = time.perf_counter() - t0
    return {"value": round(job.lattice.n * n / dt / 1e6, 3), "threads": threads, "steps": n,
            "seconds": round(dt, 2)}


def cpu_baseline(job, target_s: float = 10.0, others=()) -> dict:
    """The oracle on the headline workload on all the cores this process may use (at most 16,
    the machine's CPU share for one GPU) and on one thread; `others` (name, job) pairs are timed the
    same way, more briefly."""
    host = host_info()
    cores = max(1, min(16, host["nproc"]))
    allc = oracle_mlups(job, cores, target_s)
    one = oracle_mlups(job, 1, target_s)
    lat = job.lattice
    out = {"value": allc["value"], "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"{allc['steps']} full steps (IB + collide/stream + membrane) of the same "
                     f"{lat.nx}x{lat.ny}x{lat.nz} case after 2 steps, {allc['seconds']} s, FP64, "
                     f"OpenMP over lattice nodes on {cores} threads",
           "single_thread": {"value": one["value"], "unit": "MLUPS", "cores": 1,
                             "sample": f"{one['steps']} steps, {one['seconds']} s"},
           "host": host}
    extra = {}
    for name, j in others:
        a = oracle_mlups(j, cores, target_s / 2)
        b = oracle_mlups(j, 1, target_s / 2)
        extra[name] = {"all_cores_mlups": a["value"], "single_thread_mlups": b["value"],
                       "steps": [a["steps"], b["steps"]]}
    if extra:
        out["other_workloads"] = extra
    return out


def run_plain(api, I, torch, name: str, seed: int, steps: int, warmup: int):
    """The plain per-job form of one workload: timed steps with sampled sweep events."""
    stream = torch.cuda.current_stream()
    gen, gen_args, wl_text = WORKLOADS[name]
    job = getattr(I, gen)(*gen_args) if gen_args is not None else getattr(I, gen)(seed)
    spec = job.lattice
    s_bytes = 4 if spec.storage == I.STORE_F32 else 2
    lat = api.Lattice(spec, stream=stream)
    lat.add_body(job.body, job.xyz, job.tri)
    lat.step(warmup)
    lat.sync()
    lat.set_timing(TIMING_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat.sync()  # raises on instability / domain errors
    sweep_ms, nsweep = lat.kernel_time(0)
    step_ms, nstep = lat.kernel_time(1)
    lat.set_timing(False)
    lat.destroy()
    n = spec.n
    sweep_avg_s = sweep_ms / nsweep / 1e3
    bytes_per_launch = 2 * 19 * s_bytes * n  # algorithmic: read and write 19 stored values per node
    achieved = bytes_per_launch / sweep_avg_s / 1e9
    roof_mlups = PEAK_HBM_GBS * 1e9 / (2 * 19 * s_bytes) / 1e6
    mlups = n * steps / wall / 1e6
    return dict(job=job, spec=spec, s_bytes=s_bytes, wl_text=wl_text, gen_args=gen_args, wall=wall,
                mlups=mlups, sweep_avg_s=sweep_avg_s, nsweep=nsweep, step_ms=step_ms, nstep=nstep,
                bytes_per_launch=bytes_per_launch, achieved=achieved, roof_mlups=roof_mlups)


def plain_summary(r, steps: int) -> dict:
    n = r["spec"].n
    return {"mlups": round(r["mlups"], 2), "ms_per_step": round(r["wall"] / steps * 1e3, 5),
            "full_step_frac_of_roofline_mlups": round(r["mlups"] / r["roof_mlups"], 4),
            "sweep_us_avg": round(r["sweep_avg_s"] * 1e6, 3),
            "sweep_frac": round(r["achieved"] / PEAK_HBM_GBS, 4),
            "sweep_achieved_GBs": round(r["achieved"], 1),
            "populations_bytes": 2 * 19 * r["s_bytes"] * n,
            "lattice": [r["spec"].nx, r["spec"].ny, r["spec"].nz], "steps": steps}


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
    sweep shape) against the plain form: the same jobs one at a time with FP32 storage, each
    timed over a tenth of the batched steps (at least 10)."""
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
    roof_mlups = PEAK_HBM_GBS * 1e9 / (2 * 19 * 2) / 1e6
    return {
        "metric": METRIC, "mode": "batch",
        "value": round(nodes / per_step / 1e6, 2), "unit": "MLUPS",
        "full_step_frac_of_roofline_mlups": round(nodes / per_step / 1e6 / roof_mlups, 4),
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
    """Serving: Poisson arrivals (mean 4 jobs/s over --serve-window seconds) of capsule-shear and
    settling jobs, served by the continuous-batching server (FP16, slots sized once for the
    memory budget).  Time to result runs from each job's arrival time (not its submission);
    jobs not finished when the run stops are reported as censored with the time they had waited.
    Capacity, the jobs per hour at saturation, is measured separately by submitting a block of
    jobs at once.  The plain form is a one-slot FIFO of the same stream with FP32 storage."""
    import numpy as np
    import torch
    from paper_2207_06029_amd import api
    from paper_2207_06029_amd import inputs as I

    def run(stream_jobs, slots, storage, budget, tick, cutoff_s, label):
        srv = api.Server(hbm_budget_bytes=budget, max_slots=slots, steps_per_tick=tick,
                         storage=storage, stream=torch.cuda.current_stream())
        info = srv.info()
        pending = sorted(stream_jobs, key=lambda j: j.arrival_s)
        arrival = {j.tag: j.arrival_s for j in pending}
        t0_ns = time.monotonic_ns()   # the server stamps steady-clock (monotonic) times
        done, i, last_note = [], 0, 0.0
        while len(done) < len(pending):
            now = (time.monotonic_ns() - t0_ns) * 1e-9
            if now > cutoff_s:
                break
            if now - last_note > 10.0:
                st = srv.stats()
                print(f"[serve {label}] t={now:.0f}s submitted={i} done={len(done)} "
                      f"resident={st['resident']} queued={st['queued']}", file=sys.stderr, flush=True)
                last_note = now
            while i < len(pending) and pending[i].arrival_s <= now:
                srv.submit(pending[i])
                i += 1
            srv.tick()
            done += srv.poll()
            st = srv.stats()
            if i < len(pending) and st["resident"] == 0 and st["queued"] == 0:
                time.sleep(max(0.0, pending[i].arrival_s - (time.monotonic_ns() - t0_ns) * 1e-9))
        wall = (time.monotonic_ns() - t0_ns) * 1e-9
        st = srv.stats()
        lat = np.array([(r["t_finish_ns"] - t0_ns) * 1e-9 - arrival[r["tag"]] for r in done])
        finished = {r["tag"] for r in done}
        arrived = [j for j in pending if j.arrival_s <= wall]
        waiting = np.array([wall - j.arrival_s for j in arrived if j.tag not in finished])
        ok = sum(1 for r in done if r["status"] == 0)
        by_tag = {j.tag: j for j in pending}
        failures = []
        for r in done:
            if r["status"] != 0:
                j = by_tag[r["tag"]]
                failures.append({"tag": int(r["tag"]), "status": r["status"], "kind": j.kind,
                                 "dims": [j.lattice.nx, j.lattice.ny, j.lattice.nz], "nv": int(len(j.xyz)),
                                 "mass_ratio": round(j.body.mass_ratio, 3), "ks0": round(j.body.ks0, 5),
                                 "kb": round(j.body.kb, 6), "tau": round(j.lattice.tau, 3),
                                 "steps_done": r["steps_done"]})
        # percentiles over every arrived job, the censored ones counted as waiting forever: a
        # percentile that falls on a censored job is reported as None
        n_arr = len(arrived)
        allt = np.sort(np.concatenate([lat, np.full(len(waiting), np.inf)])) if n_arr else np.array([])
        def pct(q):
            if not n_arr:
                return None
            v = allt[min(n_arr - 1, int(np.ceil(q / 100.0 * n_arr)) - 1)]
            return None if not np.isfinite(v) else round(float(v), 3)
        return {"jobs_arrived": n_arr, "jobs_finished": len(done), "ok": ok, "failures": failures[:40],
                "censored": int(len(waiting)),
                "censored_max_wait_s": round(float(waiting.max()), 2) if len(waiting) else 0.0,
                "wall_s": round(wall, 2), "finished_per_hour": round(len(done) / wall * 3600, 1),
                "mlups": round(st["node_updates"] / wall / 1e6, 1),
                "p50_s": pct(50), "p99_s": pct(99),
                "slots": info["slots"], "slot_bytes": info["slot_bytes"], "device_bytes": info["device_bytes"]}

    budget = 32 << 30
    jobs = I.serving_stream(seed=0, rate_per_s=4.0, window_s=args.serve_window, storage=I.STORE_F16)
    served = run(jobs, slots=64, storage=I.STORE_F16, budget=budget, tick=100,
                 cutoff_s=args.serve_window * 1.5 + 30, label="served")
    capacity, cap = None, None
    if args.serve_capacity_jobs > 0:
        # capacity: a block of jobs of the same stream, all submitted at once
        block = I.serving_stream(seed=1, rate_per_s=1e6, window_s=1.0, storage=I.STORE_F16,
                                 max_jobs=args.serve_capacity_jobs)
        for j in block:
            j.arrival_s = 0.0
        cap = run(block, slots=64, storage=I.STORE_F16, budget=budget, tick=100, cutoff_s=600.0,
                  label="capacity")
        capacity = round(cap["jobs_finished"] / cap["wall_s"] * 3600, 1)
    plain, plain_window = None, min(args.serve_window, 60.0)
    if not args.serve_no_plain:
        plain = run(I.serving_stream(seed=0, rate_per_s=4.0, window_s=plain_window, storage=I.STORE_F32),
                    slots=1, storage=I.STORE_F32, budget=budget, tick=100,
                    cutoff_s=plain_window * 1.5 + 30, label="plain")
    return {"metric": METRIC, "mode": "serve", "value": capacity, "unit": "jobs/h at saturation",
            "served": served,
            "capacity": None if cap is None else {"jobs": cap["jobs_finished"], "wall_s": cap["wall_s"],
                                                  "jobs_per_hour": capacity, "mlups": cap["mlups"]},
            "offered_jobs_per_hour": 4.0 * 3600, "plain_fifo": plain,
            "config": {"workload": f"Poisson arrivals 4 jobs/s over {args.serve_window:.0f} s: "
                                   "capsule-shear and settling jobs, lattices 48^3..128x64x128, "
                                   "meshes 642-10242 vertices, 2000-10000 steps, FP16 storage, "
                                   "32 GiB budget, up to 64 slots, 100 steps per tick"
                                   + (f"; capacity from {args.serve_capacity_jobs} jobs submitted at once"
                                      if cap is not None else "")
                                   + (f"; plain FIFO over the first {plain_window:.0f} s of the stream"
                                      if plain is not None else "")},
            "dtype": "f16-storage/f32-compute", "data": "synthetic", "n_gpus": 1}


def make_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="plain mode: time only the chosen workload (no 256^3, settling and batch lines)")
    ap.add_argument("--calib-copy", type=int, default=0, help="bytes: run only a copy of that size")
    ap.add_argument("--graph", action="store_true",
                    help="also time the same steps replayed from a captured hipGraph")
    ap.add_argument("--mode", choices=["plain", "batch", "serve"], default="plain")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="prolate128",
                    help="plain mode: prolate capsule in shear at 128x64x128 (default) or 256x128x256, "
                         "or the FP16 rigid sphere settling in a 96x96x384 box")
    ap.add_argument("--serve-window", type=float, default=60.0,
                    help="serve mode: seconds of Poisson arrivals (the served run stops at 1.5x "
                         "this plus 30 s; later results are reported as censored)")
    ap.add_argument("--serve-capacity-jobs", type=int, default=256,
                    help="serve mode: jobs submitted at once to measure capacity (0: skip)")
    ap.add_argument("--serve-no-plain", action="store_true",
                    help="serve mode: skip the one-slot FIFO of the plain form")
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
    r = run_plain(api, I, torch, args.workload, args.seed, args.steps, args.warmup)
    job, spec, s_bytes = r["job"], r["spec"], r["s_bytes"]
    gen_args, wl_text = r["gen_args"], r["wl_text"]
    n = spec.n
    sweep_avg_s, nsweep, step_ms, nstep = r["sweep_avg_s"], r["nsweep"], r["step_ms"], r["nstep"]
    achieved, bytes_per_launch, wall = r["achieved"], r["bytes_per_launch"], r["wall"]
    mlups = r["mlups"]
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
                     "avg_launch_us": round(sweep_avg_s * 1e6, 3),
                     "working_set_bytes": bytes_per_launch,
                     "infinity_cache_bytes": INFINITY_CACHE_BYTES,
                     "cache_resident": bytes_per_launch <= INFINITY_CACHE_BYTES},
        "breakdown": {"sweep_us_avg": round(sweep_avg_s * 1e6, 3),
                      "sweep_launches_timed": nsweep,
                      "step_us_avg_events": round(step_ms / max(nstep, 1) * 1e3, 3),
                      "sweep_share_of_step": round(sweep_avg_s * 1e3 * nstep / max(step_ms, 1e-9), 4),
                      "sweep_only_mlups": round(n / sweep_avg_s / 1e6, 1),
                      "full_step_frac_of_roofline_mlups": round(mlups / r["roof_mlups"], 4)},
    }
    if args.graph:
        # same job as a one-job batch whose steps replay a captured hipGraph of 16 steps
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
    if not args.no_extras and args.workload == "prolate128":
        # the other measured forms of the metric, each with its own fraction of the roofline:
        # the FP32 case beyond the Infinity Cache, the FP16 rigid settling box, and the 64-job
        # batch against the same jobs one at a time
        xs = max(args.steps, EXTRA_MIN_STEPS)
        xw = max(args.warmup, EXTRA_MIN_WARMUP)
        extras = {}
        for name in ("prolate256", "settling384"):
            print(f"[bench] extra workload {name}: {xs} steps", file=sys.stderr, flush=True)
            extras[name] = plain_summary(run_plain(api, I, torch, name, args.seed, xs, xw), xs)
        print(f"[bench] extra workload batch64: {xs} steps", file=sys.stderr, flush=True)
        bargs = argparse.Namespace(**{**vars(args), "steps": xs, "warmup": xw})
        bt = bench_batch(bargs)
        extras["batch64"] = {k: bt[k] for k in ("value", "unit", "full_step_frac_of_roofline_mlups",
                                                  "jobs_per_hour", "plain_jobs_per_hour", "plain_mlups",
                                                  "ms_per_batched_step", "launch_shape")}
        extras["batch64"]["sweep_frac"] = bt["roofline"]["frac"]
        extras["batch64"]["steps"] = xs
        out["extra"] = extras
    if not args.no_cpu_baseline:
        others = () if args.no_extras else (("capsule32", I.capsule_shear_small()),
                                              ("settling384", I.settling_sphere(1.5)))
        out["cpu_baseline"] = cpu_baseline(job, others=others)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
