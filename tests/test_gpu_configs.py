"""GPU parity at the full workload sizes, in the launch configuration the benchmark uses.

The oracle runs with OpenMP on the host cores (results do not depend on the thread count)."""
import os

import numpy as np
import pytest

from paper_2207_06029_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2207_06029_amd import api as A
    return A


@pytest.fixture(scope="module", autouse=True)
def _threads(orc):
    orc.set_threads(max(1, min(16, os.cpu_count() or 1)))


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def run_both(api, orc, job, steps, storage=None):
    spec = job.lattice
    if storage is not None:
        spec.storage = storage
    lat = api.Lattice(spec)
    b = lat.add_body(job.body, job.xyz, job.tri)
    ref = orc.Lattice(spec)
    rb = ref.add_body(job.body, job.xyz, job.tri)
    lat.step(steps)
    ref.step(steps)
    lat.sync()
    _, u = lat.macros()
    _, ur = ref.macros()
    x, _ = lat.body_state(b)
    xr, _ = ref.body_state(rb)
    eu, ex = rel_l2(u, ur), rel_l2(x, xr)
    ed = rel_l2(x - job.xyz, xr - job.xyz)
    fv, F, M = lat.body_forces(b)
    fvr, Fr, Mr = ref.body_forces(rb)
    ef = rel_l2(np.concatenate([F, M]), np.concatenate([Fr, Mr]))
    print(f"  force/torque totals rel-L2 {ef:.3e} (F {F}, M {M}); vertex forces {rel_l2(fv, fvr):.3e}")
    assert ef < 1e-3
    print(f"{job.name} storage {spec.storage}: {steps} steps, rel-L2 u* {eu:.3e}, positions {ex:.3e}, "
          f"displacement {ed:.3e}")
    return eu, ex


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_prolate_shear_fp32_1000_steps(api, orc, seed):
    eu, ex = run_both(api, orc, I.prolate_shear(seed), 1000)
    assert eu < 1e-5 and ex < 1e-5


def test_settling_full_size_fp32(api, orc):
    eu, ex = run_both(api, orc, I.settling_sphere(2.0, I.STORE_F32), 100)
    assert eu < 1e-5 and ex < 1e-5


def test_settling_full_size_fp16(api, orc):
    eu, ex = run_both(api, orc, I.settling_sphere(2.0, I.STORE_F16), 100)
    assert eu < 1e-3 and ex < 1e-3
