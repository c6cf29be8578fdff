"""Batching and serving on the GPU: every job's result is bitwise the same alone and inside a
batch or the server's mix, launch shapes and graph replay do not change results, and batched
jobs match the FP64 oracle within the reduced-precision tolerance."""
import os

import numpy as np
import pytest

from paper_2207_06029_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2207_06029_amd import api as A
    return A


def mixed_jobs(n=5, steps=120):
    jobs = I.capsule_batch(seed=3, njobs=n, storage=I.STORE_F16, steps=steps)
    # add a settling job (rigid body, closed box) to the mix
    lat = I.LatticeSpec(32, 32, 48, 0.7, storage=I.STORE_F16, **I.closed_box())
    body = I.BodySpec(rigid=1, ks0=0.0, kb=0.0, kv=0.0, mass_ratio=2.0, gravity=(0.0, 0.0, -1e-4))
    xyz, tri = I.spheroid_mesh(3, (4.0, 4.0, 4.0), (15.5, 15.5, 30.0))
    jobs.append(I.Job("settle", lat, body, xyz, tri, steps, tag=99, kind="settling"))
    return jobs


def state_of(lat):
    _, u = lat.macros()
    x, _ = lat.body_state(0)
    return u, x


def test_batch_alone_vs_mix_bitwise(api):
    """Each job alone (the single-body kernel instantiations, body record in the kernel
    arguments) against the same job in a six-body mix (block tables): bit for bit, membranes
    and the rigid sphere alike."""
    jobs = mixed_jobs()
    steps = 120
    mix = api.Batch(jobs, storage=I.STORE_F16)
    mix.step(steps)
    mix.sync()
    for j, job in enumerate(jobs):
        alone = api.Batch([job], storage=I.STORE_F16)
        alone.step(steps)
        alone.sync()
        u_m, x_m = state_of(mix.lattice(j))
        u_a, x_a = state_of(alone.lattice(0))
        np.testing.assert_array_equal(u_m, u_a)
        np.testing.assert_array_equal(x_m, x_a)


def test_launch_shape_and_graph_do_not_change_results(api, tmp_path):
    jobs = mixed_jobs(3, 60)
    ref = api.Batch(jobs, storage=I.STORE_F16)
    ref.step(61)
    tuned = api.Batch(jobs, storage=I.STORE_F16, autotune=True,
                      tune_cache=str(tmp_path / "tune.txt"), use_graph=True)
    tuned.step(61)
    print("autotuned launch shape", tuned.launch_shape())
    for j in range(len(jobs)):
        u_r, x_r = state_of(ref.lattice(j))
        u_t, x_t = state_of(tuned.lattice(j))
        np.testing.assert_array_equal(u_r, u_t)
        np.testing.assert_array_equal(x_r, x_t)
    # the cache is reused by a second batch of the same shapes
    again = api.Batch(jobs, storage=I.STORE_F16, autotune=True, tune_cache=str(tmp_path / "tune.txt"))
    assert again.launch_shape() == tuned.launch_shape()


def test_batched_jobs_match_oracle(api, orc):
    orc.set_threads(max(1, min(16, os.cpu_count() or 1)))
    jobs = mixed_jobs(3, 200)
    mix = api.Batch(jobs, storage=I.STORE_F16)
    mix.step(200)
    mix.sync()
    for j in (0, len(jobs) - 1):
        job = jobs[j]
        ref = orc.Lattice(job.lattice)
        rb = ref.add_body(job.body, job.xyz, job.tri)
        ref.step(200)
        _, ur = ref.macros()
        xr, _ = ref.body_state(rb)
        u, x = state_of(mix.lattice(j))
        eu = np.linalg.norm(u - ur) / np.linalg.norm(ur)
        ex = np.linalg.norm(x - xr) / np.linalg.norm(xr)
        print(f"job {job.name}: rel-L2 u* {eu:.3e}, positions {ex:.3e}")
        assert eu < 1e-3 and ex < 1e-3


def test_server_results_match_alone(api):
    jobs = mixed_jobs(4, 0)
    for k, job in enumerate(jobs):
        job.steps = 40 + 23 * k           # uneven run lengths: jobs retire at different ticks
    srv = api.Server(hbm_budget_bytes=1 << 34, max_slots=3, steps_per_tick=16, storage=I.STORE_F16)
    ids = {srv.submit(job): job for job in jobs}
    results = {}
    for _ in range(100):
        srv.tick()
        for r in srv.poll(with_positions=True):
            results[r["id"]] = r
        if len(results) == len(jobs):
            break
    assert len(results) == len(jobs)
    for jid, job in ids.items():
        r = results[jid]
        assert r["status"] == 0 and r["steps_done"] == job.steps
        alone = api.Batch([job], storage=I.STORE_F16)
        alone.step(job.steps)
        x_a, _ = alone.lattice(0).body_state(0)
        np.testing.assert_array_equal(r["xyz"], x_a)


def test_server_alone_vs_mix_24_stream_jobs(api):
    """24 jobs from the serving-stream generator (capsule-shear and settling, uneven sizes and
    run lengths) served with 8 slots: every result equals the same job run alone, bitwise."""
    jobs = I.serving_stream(seed=7, rate_per_s=1e6, window_s=1.0, storage=I.STORE_F16,
                            steps_range=(40, 200), levels=(2, 3),
                            lattices=((32, 32, 32), (40, 32, 40), (48, 48, 48)), max_jobs=24)
    assert len(jobs) == 24 and {j.kind for j in jobs} == {"shear", "settling"}
    srv = api.Server(hbm_budget_bytes=1 << 34, max_slots=8, steps_per_tick=24, storage=I.STORE_F16)
    ids = {srv.submit(job): job for job in jobs}
    results = {}
    for _ in range(400):
        srv.tick()
        for r in srv.poll(with_positions=True):
            results[r["id"]] = r
        if len(results) == len(jobs):
            break
    assert len(results) == len(jobs)
    for jid, job in ids.items():
        r = results[jid]
        assert r["status"] == 0 and r["steps_done"] == job.steps, (job.name, r["status"])
        alone = api.Batch([job], storage=I.STORE_F16)
        alone.step(job.steps)
        x_a, _ = alone.lattice(0).body_state(0)
        np.testing.assert_array_equal(r["xyz"], x_a)
        alone.destroy()


def test_server_splices_jobs_without_allocating(api):
    """Admissions and retirements write the slot's table entries and state in place: the
    server's device memory is fixed at creation, slots are reused after a retirement, and every
    job still ends bitwise like the same job run alone."""
    jobs = I.serving_stream(seed=11, rate_per_s=1e6, window_s=1.0, storage=I.STORE_F16,
                            steps_range=(30, 90), levels=(2, 3),
                            lattices=((32, 32, 32), (40, 32, 40)), max_jobs=10)
    srv = api.Server(hbm_budget_bytes=1 << 34, max_slots=3, steps_per_tick=20, storage=I.STORE_F16,
                     slot_vertices=2562)
    info = srv.info()
    assert info["slots"] == 3 and info["device_bytes"] > 3 * 2 * 19 * 2 * 128 * 64 * 128
    ids = {srv.submit(job): job for job in jobs}
    results, max_res = {}, 0
    for _ in range(200):
        srv.tick()
        max_res = max(max_res, srv.stats()["resident"])
        assert srv.info()["device_bytes"] == info["device_bytes"]
        for r in srv.poll(with_positions=True):
            results[r["id"]] = r
        if len(results) == len(jobs):
            break
    assert len(results) == len(jobs) and max_res == 3
    for jid, job in ids.items():
        r = results[jid]
        assert r["status"] == 0 and r["steps_done"] == job.steps
        alone = api.Batch([job], storage=I.STORE_F16)
        alone.step(job.steps)
        x_a, _ = alone.lattice(0).body_state(0)
        np.testing.assert_array_equal(r["xyz"], x_a)
        alone.destroy()


def _tune_key(jobs, storage):
    """The tune cache's key of a job mix: storage, then each lattice shape with its count."""
    cnt = {}
    for j in jobs:
        k = f"{j.lattice.nx}x{j.lattice.ny}x{j.lattice.nz}"
        cnt[k] = cnt.get(k, 0) + 1
    return f"s{storage}" + "".join(f";{k}*{v}" for k, v in sorted(cnt.items()))


def test_xcd_tile_order_does_not_change_results(api, tmp_path):
    """The sweep's XCD chunking only reorders tiles: dispatch order and chunks of 8 and 3 give
    bitwise the same state.  The shapes are forced through the tune cache."""
    jobs = mixed_jobs(3, 40)
    key = _tune_key(jobs, I.STORE_F16)
    states = []
    for chunk in (0, 8, 3):
        cache = tmp_path / f"tune{chunk}.txt"
        cache.write_text(f"{key} 256 1 {chunk}\n")
        bt = api.Batch(jobs, storage=I.STORE_F16, autotune=True, tune_cache=str(cache))
        assert bt.launch_shape() == (256, 1)
        bt.step(40)
        states.append([state_of(bt.lattice(j)) for j in range(len(jobs))])
        bt.destroy()
    for other in states[1:]:
        for (u_r, x_r), (u_o, x_o) in zip(states[0], other):
            np.testing.assert_array_equal(u_r, u_o)
            np.testing.assert_array_equal(x_r, x_o)


def test_tune_cache_lines_without_chunk_still_load(api, tmp_path):
    jobs = mixed_jobs(2, 10)
    cache = tmp_path / "old.txt"
    cache.write_text(f"{_tune_key(jobs, I.STORE_F16)} 512 2\n")
    bt = api.Batch(jobs, storage=I.STORE_F16, autotune=True, tune_cache=str(cache))
    assert bt.launch_shape() == (512, 2)
    bt.step(10)
    bt.sync()
