"""Serving policy on the CPU: the server in dry-run mode schedules (FIFO admission into the slots
that the device-memory budget holds, lock-step ticks that never overshoot a job's run length,
retirement, time-to-result stamps) without touching a GPU."""
import numpy as np
import pytest

from paper_2207_06029_amd import inputs as I


@pytest.fixture(scope="module")
def api():
    from paper_2207_06029_amd import api as A
    return A


def small_job(steps, tag, edge=24):
    rng = np.random.default_rng(tag)
    spec = I.LatticeSpec(edge, edge, edge, 0.8, storage=I.STORE_F16, **I.shear_walls(0.01))
    body = I.BodySpec(rigid=0, ks0=0.01, kb=0.001, kv=0.0, mass_ratio=1.0)
    xyz, tri = I.spheroid_mesh(2, (4.0, 4.0, 4.0), ((edge - 1) / 2,) * 3, I.uniform_rotation(rng))
    return I.Job(f"j{tag}", spec, body, xyz, tri, steps, tag=tag)


def test_admission_respects_slots_and_fifo(api):
    srv = api.Server(hbm_budget_bytes=1 << 40, max_slots=2, steps_per_tick=10, dry_run=True)
    ids = [srv.submit(small_job(s, t)) for t, s in enumerate([30, 10, 20, 10])]
    order = []
    max_res = 0
    for _ in range(20):
        srv.tick()
        st = srv.stats()
        max_res = max(max_res, st["resident"])
        order += [r["id"] for r in srv.poll()]
    assert max_res == 2
    assert sorted(order) == sorted(ids)
    # job 1 (10 steps) finishes first; jobs admitted FIFO, so job 2 starts before job 3
    assert order[0] == ids[1]
    assert srv.stats()["queued"] == 0 and srv.stats()["resident"] == 0


def test_ticks_never_overshoot_run_length(api):
    srv = api.Server(hbm_budget_bytes=1 << 40, max_slots=8, steps_per_tick=64, dry_run=True)
    steps = [5, 64, 100, 129, 1]
    for t, s in enumerate(steps):
        srv.submit(small_job(s, t))
    done = {}
    for _ in range(20):
        srv.tick()
        for r in srv.poll():
            done[r["tag"]] = r["steps_done"]
    assert done == {t: s for t, s in enumerate(steps)}


def test_memory_budget_admission(api):
    one = small_job(1000, 0)      # stays resident after one tick
    probe = api.Server(hbm_budget_bytes=1 << 40, max_slots=8, steps_per_tick=10, dry_run=True,
                       slot_nodes=32 ** 3, slot_vertices=642)
    probe.submit(one)
    probe.tick()
    per_job = probe.stats()["resident_bytes"]
    assert per_job == probe.info()["slot_bytes"]
    assert per_job > 2 * 19 * 32 ** 3 * 2          # both population buffers of a slot
    assert probe.info()["slots"] == 8 and probe.info()["device_bytes"] == 0
    # a budget for two slots: never more than two resident, the rest wait
    srv = api.Server(hbm_budget_bytes=2 * per_job + 1, max_slots=8, steps_per_tick=5, dry_run=True,
                     slot_nodes=32 ** 3, slot_vertices=642)
    assert srv.info()["slots"] == 2
    for t in range(5):
        srv.submit(small_job(10, t))
    seen = 0
    for _ in range(30):
        srv.tick()
        st = srv.stats()
        assert st["resident"] <= 2 and st["resident_bytes"] <= 2 * per_job + 1
        seen += len(srv.poll())
    assert seen == 5


def test_job_that_never_fits_is_rejected(api):
    # a budget that holds no slot
    srv = api.Server(hbm_budget_bytes=1 << 20, max_slots=4, steps_per_tick=10, dry_run=True)
    with pytest.raises(api.L.LbibError) as ei:
        srv.submit(small_job(10, 0))
    assert ei.value.code == -2
    # a job larger than the slots
    srv = api.Server(hbm_budget_bytes=1 << 40, max_slots=4, steps_per_tick=10, dry_run=True,
                     slot_nodes=16 ** 3)
    with pytest.raises(api.L.LbibError) as ei:
        srv.submit(small_job(10, 0))
    assert ei.value.code == -2


def test_continuous_batching_admits_while_others_run(api):
    srv = api.Server(hbm_budget_bytes=1 << 40, max_slots=4, steps_per_tick=10, dry_run=True)
    long_id = srv.submit(small_job(200, 0))
    srv.tick()
    late = srv.submit(small_job(20, 1))
    srv.tick()
    assert srv.stats()["resident"] == 2          # admitted while the long job is running
    got = []
    for _ in range(30):
        srv.tick()
        got += srv.poll()
    first = got[0]
    assert first["id"] == late and first["t_admit_ns"] >= first["t_submit_ns"]
    assert got[-1]["id"] == long_id
    assert all(r["t_finish_ns"] >= r["t_admit_ns"] for r in got)


def test_bad_jobs_rejected_at_submit(api):
    srv = api.Server(hbm_budget_bytes=1 << 40, max_slots=4, steps_per_tick=10, dry_run=True)
    j = small_job(10, 0)
    j.tri = j.tri[:-1]                      # open surface
    with pytest.raises(api.L.LbibError):
        srv.submit(j)
    j = small_job(10, 1)
    j.lattice.tau = 0.5
    with pytest.raises(api.L.LbibError):
        srv.submit(j)
