"""Full-size parity against stored oracle results (tests/golden/*.npz, written by
tests/golden/make_oracle_goldens.py, which runs only the FP64 oracle): the settling box at every
density ratio of the precision case, and three jobs of the seed-0 64-job capsule batch over
their whole run, stepped inside the full batch in the launch configuration the benchmark times
(FP16 storage, autotuned sweep shape, hipGraph replay).  Compared: u* at the stored node sample,
vertex positions and displacements, force and torque totals."""
import os

import numpy as np
import pytest

from paper_2207_06029_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def api():
    from paper_2207_06029_amd import api as A
    return A


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.fail(f"{name} missing: run tests/golden/make_oracle_goldens.py")
    return dict(np.load(path, allow_pickle=False))


def compare(lat, b, ref, xyz0, label):
    _, u = lat.macros()
    x, _ = lat.body_state(b)
    _, F, M = lat.body_forces(b)
    idx = ref["idx"]
    eu = rel_l2(u[:, idx], ref["u"])
    ex = rel_l2(x, ref["xyz"])
    ed = rel_l2(x - xyz0, ref["xyz"] - xyz0)
    ef = rel_l2(np.concatenate([F, M]), np.concatenate([ref["F"], ref["M"]]))
    print(f"{label}: rel-L2 u* (sampled) {eu:.3e}, positions {ex:.3e}, displacement {ed:.3e}, "
          f"force/torque {ef:.3e}")
    return eu, ex, ed, ef


@pytest.mark.parametrize("ratio", I.SETTLING_DENSITY_RATIOS)
def test_settling_every_density_ratio_fp16(api, ratio):
    """96x96x384 settling box, FP16 shifted storage, 1000 steps: within the 1e-3
    reduced-precision gate of the oracle at each density ratio of the precision case."""
    ref = load(f"settling_ratio{ratio:g}_1000.npz")
    job = I.settling_sphere(ratio, I.STORE_F16)
    lat = api.Lattice(job.lattice)
    b = lat.add_body(job.body, job.xyz, job.tri)
    lat.step(int(ref["steps"]))
    lat.sync()
    eu, ex, ed, ef = compare(lat, b, ref, job.xyz, f"settling ratio {ratio} FP16")
    assert eu < 1e-3 and ex < 1e-3 and ed < 1e-3 and ef < 1e-3


def test_batch64_jobs_over_their_whole_run(api):
    """Jobs 2, 5 and 17 of the seed-0 64-job batch (32^3 level 4, 64^3 level 3 with the mass
    floor, 96^3 level 4), 2000 steps inside the full FP16 batch: within 1e-3 of the oracle."""
    jobs = I.capsule_batch(seed=0, njobs=64, storage=I.STORE_F16, steps=2000)
    bt = api.Batch(jobs, storage=I.STORE_F16, autotune=True, use_graph=True)
    refs = {j: load(f"batch64_seed0_job{j}.npz") for j in (2, 5, 17)}
    steps = int(refs[2]["steps"])
    assert all(int(r["steps"]) == steps for r in refs.values())
    bt.step(steps)
    bt.sync()
    for j, ref in refs.items():
        eu, ex, ed, ef = compare(bt.lattice(j), 0, ref, jobs[j].xyz, f"batch64 job {j}")
        assert eu < 1e-3 and ex < 1e-3 and ed < 1e-3
