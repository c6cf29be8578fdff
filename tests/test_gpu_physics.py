"""Closed-form physics checks of the GPU path (no oracle: these runs are far beyond its reach).

Jeffery orbit (Sec. 2.3): a neutrally buoyant rigid prolate spheroid of aspect ratio r whose
axis lies in the flow-gradient plane of a simple shear flow of rate gamma turns by pi in
T = pi (r + 1/r) / gamma at vanishing Reynolds number; for r = 2, T gamma = 7.854 (the paper
measures 7.853).
"""
import math

import numpy as np
import pytest

from paper_2207_06029_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2207_06029_amd import api as A
    return A


def _crossing(ts, phis, target):
    """First time the unwrapped angle falls through `target` (linear interpolation)."""
    for k in range(1, len(phis)):
        if phis[k - 1] > target >= phis[k]:
            w = (phis[k - 1] - target) / (phis[k - 1] - phis[k])
            return ts[k - 1] + w * (ts[k] - ts[k - 1])
    return None


def test_jeffery_orbit_rigid_prolate(api):
    n = 96
    a, b = 8.0, 4.0
    tau = 1.0
    nu = (tau - 0.5) / 3.0
    re = 0.05                                  # Re = gamma a^2 / nu
    gamma = re * nu / (a * a)
    u_wall = gamma * (n - 1) / 2.0
    spec = I.LatticeSpec(n, n, n, tau, **I.shear_walls(u_wall))
    lat = api.Lattice(spec)
    # start from the linear shear profile u_x = gamma (y - (n-1)/2); node index x + n (y + n z)
    _, yy, _ = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    u = np.zeros((3, n ** 3))
    u[0] = gamma * (yy.reshape(-1) - (n - 1) / 2.0)
    lat.init(np.ones(n ** 3), u)
    phi0 = math.pi / 4
    c, s = math.cos(phi0), math.sin(phi0)
    rot = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    centre = np.array([(n - 1) / 2.0] * 3)
    xyz, tri = I.spheroid_mesh(4, (a, b, b), centre, rot)
    tip = int(np.argmax((xyz - centre) @ rot[:, 0]))
    body = I.BodySpec(rigid=1, ks0=0.0, kb=0.0, kv=0.0, mass_ratio=1.0)
    bid = lat.add_body(body, xyz, tri)
    every = 200
    half = math.pi * (2.0 + 0.5) / gamma        # expected steps per half turn
    total = int(2.0 * half)
    d0 = xyz[tip] - xyz.mean(axis=0)
    ts, phis = [0.0], [math.atan2(d0[1], d0[0])]
    for k in range(1, total // every + 1):
        lat.step(every)
        pos, _ = lat.body_state(bid)
        d = pos[tip] - pos.mean(axis=0)
        ang = math.atan2(d[1], d[0])
        # unwrap against the previous sample
        prev = phis[-1]
        ang += 2 * math.pi * round((prev - ang) / (2 * math.pi))
        ts.append(k * every)
        phis.append(ang)
    t1 = _crossing(ts, phis, -math.pi / 2)
    t2 = _crossing(ts, phis, -3 * math.pi / 2)
    assert t1 is not None and t2 is not None, f"no full half turn: final angle {phis[-1]:.3f}"
    period = (t2 - t1) * gamma
    print(f"Jeffery half period T*gamma = {period:.4f} (closed form {math.pi * 2.5:.4f}), "
          f"gamma {gamma:.3e}, Re {re}, {total} steps")
    assert abs(period - math.pi * 2.5) / (math.pi * 2.5) < 0.01
