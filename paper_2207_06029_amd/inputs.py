"""Seeded synthetic inputs for the LB / dynamic-IB capsule solver.

This module only *generates problem data*: closed triangulated surfaces
(subdivided icosahedra and spheroids), random orientations, random smooth
initial fields, and the job descriptions of the workloads the solver is
measured on.  It holds none of the scheme's arithmetic (no equilibria,
no forcing, no MLS, no membrane mechanics); both the FP64 CPU oracle and
the HIP path consume exactly the same arrays produced here.

Workload shapes follow the paper's cases: a spherical capsule in simple
shear (Sec. 2, capsule-in-shear validation), a prolate membrane tumbling in
shear (Sec. 2, deformable prolate study), and a rigid sphere settling under
gravity in a closed box (Sec. 2, settling-sphere validation).  Meshes use
markers on triangle centroids (Sec. 1.2, Fig. IB a).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

# boundary kinds per face, same integers the C interfaces use
BC_PERIODIC = 0
BC_ZOUHE_VELOCITY = 1
BC_BOUNCEBACK = 2

STORE_F32 = 0
STORE_F16 = 1
STORE_BF16 = 2

INTEGRATOR_DISPLACEMENT = 0   # membrane position by Eq. verletPos, velocity = step displacement
INTEGRATOR_PAPER = 1          # the printed three-stage verletPos / verletVel / verletPos update
INTEGRATOR_KINEMATIC = 2      # kinematic IB: points advected with the interpolated fluid velocity

# ---------------------------------------------------------------- meshes


def icosphere(level: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit sphere from a regular icosahedron subdivided `level` times.

    Returns (xyz float64[nv,3], tri int32[nt,3]) with counter-clockwise
    winding seen from outside.  nv = 10*4**level + 2, nt = 20*4**level.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    # orient every base face outward
    tris = []
    for a, b, c in faces:
        n = np.cross(verts[b] - verts[a], verts[c] - verts[a])
        if np.dot(n, verts[a] + verts[b] + verts[c]) < 0.0:
            b, c = c, b
        tris.append((a, b, c))
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            k = cache.get(key)
            if k is None:
                p = verts[i] + verts[j]
                verts.append(p / np.linalg.norm(p))
                k = len(verts) - 1
                cache[key] = k
            return k

        nxt = []
        for a, b, c in tris:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nxt += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        tris = nxt
    return np.array(verts, dtype=np.float64), np.array(tris, dtype=np.int32)


def uniform_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation matrix from a normalised 4-D Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def spheroid_mesh(level: int, semi_axes: Sequence[float], centre: Sequence[float],
                  rotation: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Icosphere scaled to semi-axes (a, b, c) along body x, y, z, rotated, then moved."""
    xyz, tri = icosphere(level)
    xyz = xyz * np.asarray(semi_axes, dtype=np.float64)[None, :]
    if rotation is not None:
        xyz = xyz @ np.asarray(rotation, dtype=np.float64).T
    return xyz + np.asarray(centre, dtype=np.float64)[None, :], tri


# ---------------------------------------------------------------- job data


@dataclass
class LatticeSpec:
    nx: int
    ny: int
    nz: int
    tau: float
    bc: Tuple[int, int, int, int, int, int] = (0, 0, 0, 0, 0, 0)  # -x,+x,-y,+y,-z,+z
    wall_u: Tuple[Tuple[float, float, float], ...] = ((0.0, 0.0, 0.0),) * 6
    body_force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    storage: int = STORE_F32

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class BodySpec:
    rigid: int
    ks0: float
    kb: float
    kv: float
    mass_ratio: float
    thickness: float = 1.0
    gravity: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    mls_rw: float = 1.3
    mls_alpha: float = 0.3
    probe_len: float = 1.2
    shell_h: float = 1.0
    integrator: int = INTEGRATOR_DISPLACEMENT


@dataclass
class Job:
    name: str
    lattice: LatticeSpec
    body: Optional[BodySpec]
    xyz: Optional[np.ndarray]
    tri: Optional[np.ndarray]
    steps: int
    tag: int = 0
    kind: str = "shear"
    arrival_s: float = 0.0
    drawn_mass_ratio: Optional[float] = None


def shear_walls(u_wall: float) -> dict:
    """Zou-He velocity walls on the y faces moving at -u_wall / +u_wall along x; x, z periodic."""
    return dict(bc=(BC_PERIODIC, BC_PERIODIC, BC_ZOUHE_VELOCITY, BC_ZOUHE_VELOCITY,
                    BC_PERIODIC, BC_PERIODIC),
                wall_u=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (-u_wall, 0.0, 0.0),
                        (u_wall, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0)))


def closed_box() -> dict:
    """Halfway bounce-back no-slip walls on all six faces."""
    return dict(bc=(BC_BOUNCEBACK,) * 6, wall_u=((0.0, 0.0, 0.0),) * 6)


def lid_cavity(u_lid: float) -> dict:
    """Closed box of Zou-He velocity walls: the high-y wall (the lid) slides along +z at u_lid,
    the other five rest (the lid-driven cavity of Sec. 2.1)."""
    wall_u = [(0.0, 0.0, 0.0)] * 6
    wall_u[3] = (0.0, 0.0, float(u_lid))
    return dict(bc=(BC_ZOUHE_VELOCITY,) * 6, wall_u=tuple(wall_u))


def cavity_spec(n: int, reynolds: float, tau: float = 1.0, storage: int = STORE_F32) -> LatticeSpec:
    """Lid-driven cube of n nodes per side, walls on the first and last nodes (side L = n - 1):
    lid speed from Re = u L / nu with nu = (tau - 1/2) / 3 (Sec. 2.1 keeps tau = 1)."""
    nu = (tau - 0.5) / 3.0
    u = reynolds * nu / (n - 1)
    return LatticeSpec(n, n, n, tau, storage=storage, **lid_cavity(u))


# Rigid bodies this many times denser than the fluid, without gravity, stand still to within
# F t^2 / (2 m): a fixed obstacle for the dynamic immersed boundary.
FIXED_BODY_MASS_RATIO = 1e9


def cavity_sphere_job(n: int, reynolds: float, level: int, tau: float = 1.0,
                      storage: int = STORE_F32, steps: int = 0) -> "Job":
    """The lid-driven cavity with a fixed solid sphere of diameter 0.2 L at its centre
    (Sec. 2.1, second experiment; L = n - 1).  Mesh level chosen by the caller: levels 3, 4
    and 5 at L = 48, 96 and 192 keep about 4.4 markers per unit area."""
    lat = cavity_spec(n, reynolds, tau=tau, storage=storage)
    L = n - 1
    radius = 0.1 * L
    c = 0.5 * L
    xyz, tri = spheroid_mesh(level, (radius, radius, radius), (c, c, c))
    body = BodySpec(rigid=1, ks0=0.0, kb=0.0, kv=0.0, mass_ratio=FIXED_BODY_MASS_RATIO)
    return Job(f"cavity_sphere_n{n}", lat, body, xyz, tri, steps, kind="cavity")


def square_duct(u_wall: float = 0.0) -> dict:
    """Zou-He walls on the y and z faces, periodic along x; every wall slides along x at u_wall."""
    return dict(bc=(BC_PERIODIC, BC_PERIODIC) + (BC_ZOUHE_VELOCITY,) * 4,
                wall_u=((0.0, 0.0, 0.0),) * 2 + ((float(u_wall), 0.0, 0.0),) * 4)


def duct_poiseuille(y, z, width: float, accel: float, nu: float, terms: int = 200) -> np.ndarray:
    """Fully developed flow along x in a square duct of side `width` (walls at 0 and width in y
    and z) driven by a uniform acceleration: the Fourier-series solution of
    nu (u_yy + u_zz) = -accel with u = 0 on the walls."""
    a = 0.5 * width
    yc = np.asarray(y, dtype=np.float64) - a
    zc = np.asarray(z, dtype=np.float64) - a
    u = np.zeros(np.broadcast(yc, zc).shape)
    for j in range(terms):
        n = 2 * j + 1
        k = n * np.pi / (2.0 * a)
        # cosh(k z) / cosh(k a), written with exponentials that cannot overflow
        ratio = (np.exp(k * (np.abs(zc) - a)) + np.exp(-k * (np.abs(zc) + a))) / (1.0 + np.exp(-2.0 * k * a))
        u += (-1.0) ** j / n ** 3 * (1.0 - ratio) * np.cos(k * yc)
    return 16.0 * a * a * accel / (nu * np.pi ** 3) * u


def ks0_from_capillary(ca: float, tau: float, shear_rate: float, radius: float,
                       rho: float = 1.0) -> float:
    """Global spring constant from the capillary number Ca = rho*nu*u_ref/k_s0 (Sec. 1.3,
    network model), with u_ref = shear_rate*radius and the lattice viscosity nu=(tau-1/2)/3."""
    nu = (tau - 0.5) / 3.0
    return rho * nu * shear_rate * radius / ca


def capsule_shear_small() -> Job:
    """32^3 box, tau=0.8, x/z periodic, Zou-He walls on y=0 / y=31 moving at -/+0.01 along x.
    Spherical capsule R=6 at the box centre, level-3 icosphere (642 nodes, 1280 triangles),
    k_s0=0.01, k_b=0.001, neutrally buoyant; 1000 steps from rest, no randomness."""
    lat = LatticeSpec(32, 32, 32, 0.8, **shear_walls(0.01))
    body = BodySpec(rigid=0, ks0=0.01, kb=0.001, kv=0.0, mass_ratio=1.0)
    xyz, tri = spheroid_mesh(3, (6.0, 6.0, 6.0), (15.5, 15.5, 15.5))
    return Job("capsule_shear_32", lat, body, xyz, tri, 1000)


def prolate_shear(seed: int) -> Job:
    """128x64x128 box, tau~U(0.6,1.0), wall shear rate 1e-4/step (walls at y=0, 63).
    Prolate spheroid capsule a=12, b=c=6, level-4 mesh (2562 nodes), random orientation;
    Ca=0.05 (u_ref = shear_rate*a), k_b = 0.01*k_s0; 5000 steps."""
    rng = np.random.default_rng(seed)
    tau = float(rng.uniform(0.6, 1.0))
    rot = uniform_rotation(rng)
    shear = 1e-4
    ny = 64
    lat = LatticeSpec(128, ny, 128, tau, **shear_walls(shear * (ny - 1) / 2.0))
    ks0 = ks0_from_capillary(0.05, tau, shear, 12.0)
    body = BodySpec(rigid=0, ks0=ks0, kb=0.01 * ks0, kv=0.0, mass_ratio=1.0)
    xyz, tri = spheroid_mesh(4, (12.0, 6.0, 6.0), (63.5, 31.5, 63.5), rot)
    return Job(f"prolate_shear_s{seed}", lat, body, xyz, tri, 5000, tag=seed)


def prolate_shear_large(seed: int) -> Job:
    """Same physics as prolate_shear at twice the linear size: 256x128x256, a=24, level 5."""
    rng = np.random.default_rng(seed)
    tau = float(rng.uniform(0.6, 1.0))
    rot = uniform_rotation(rng)
    shear = 0.5e-4
    ny = 128
    lat = LatticeSpec(256, ny, 256, tau, **shear_walls(shear * (ny - 1) / 2.0))
    ks0 = ks0_from_capillary(0.05, tau, shear, 24.0)
    body = BodySpec(rigid=0, ks0=ks0, kb=0.01 * ks0, kv=0.0, mass_ratio=1.0)
    xyz, tri = spheroid_mesh(5, (24.0, 12.0, 12.0), (127.5, 63.5, 127.5), rot)
    return Job(f"prolate_shear_large_s{seed}", lat, body, xyz, tri, 5000, tag=seed)


SETTLING_DENSITY_RATIOS = (1.1, 1.5, 2.0, 4.0, 8.0)


def settling_sphere(density_ratio: float = 1.5, storage: int = STORE_F16) -> Job:
    """96x96x384 closed box (halfway bounce-back), tau=0.7, rigid sphere R=8 (level 4)
    released at rest 2.67 diameters below the lid, gravity 1e-5 along -z; 20000 steps."""
    lat = LatticeSpec(96, 96, 384, 0.7, storage=storage, **closed_box())
    body = BodySpec(rigid=1, ks0=0.0, kb=0.0, kv=0.0, mass_ratio=float(density_ratio),
                    gravity=(0.0, 0.0, -1e-5))
    xyz, tri = spheroid_mesh(4, (8.0, 8.0, 8.0), (47.5, 47.5, 340.0))
    return Job(f"settling_rho{density_ratio:g}", lat, body, xyz, tri, 20000, kind="settling")


# Capillary numbers of the generated membranes, log-uniform: from the stiffest of the paper's
# deformable cases (G = 0.01, prolate tumbling study) to strongly deforming capsules (0.5).
CA_RANGE = (0.01, 0.5)


def _shear_job(rng: np.random.Generator, dims: Tuple[int, int, int], level: int,
               storage: int, steps: int, name: str, tag: int) -> Job:
    nx, ny, nz = dims
    tau = float(rng.uniform(0.6, 1.0))
    u_wall = 0.01
    shear = 2.0 * u_wall / (ny - 1)
    radius = 0.2 * min(dims)
    oblate = bool(rng.uniform() < 0.5)
    semi = (radius, radius, 0.5 * radius) if oblate else (radius, radius, radius)
    rot = uniform_rotation(rng)
    ca = float(math.exp(rng.uniform(math.log(CA_RANGE[0]), math.log(CA_RANGE[1]))))
    kb_ratio = float(rng.uniform(0.0, 0.05))
    drawn_ratio = float(rng.uniform(0.0, 2.0))
    ks0 = ks0_from_capillary(ca, tau, shear, radius)
    lat = LatticeSpec(nx, ny, nz, tau, storage=storage, **shear_walls(u_wall))
    centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    xyz, tri = spheroid_mesh(level, semi, centre, rot)
    mass_ratio = max(drawn_ratio, membrane_mass_floor(ks0, xyz, tri))
    body = BodySpec(rigid=0, ks0=ks0, kb=kb_ratio * ks0, kv=0.0, mass_ratio=mass_ratio)
    job = Job(name, lat, body, xyz, tri, steps, tag=tag, kind="shear")
    job.drawn_mass_ratio = drawn_ratio
    return job


def membrane_mass_floor(ks0: float, xyz: np.ndarray, tri: np.ndarray) -> float:
    """Smallest solid/fluid density ratio given to a generated membrane job: 0.5, and at least
    2 k_s0 / (mean triangle area).  Lighter membranes (ratio 0.1 and 0.2 in the batching mix)
    diverge under the weakly coupled explicit vertex update, and so do stiff, finely meshed
    ones below about k_s0 / (mean area); the draws are floored so every job runs."""
    a = xyz[tri[:, 1]] - xyz[tri[:, 0]]
    b = xyz[tri[:, 2]] - xyz[tri[:, 0]]
    area = 0.5 * np.linalg.norm(np.cross(a, b), axis=1).mean()
    return max(0.5, 2.0 * ks0 / area)


BATCH_EDGES = (32, 48, 64, 80, 96)


def capsule_batch(seed: int = 0, njobs: int = 64, storage: int = STORE_F16,
                  steps: int = 2000) -> List[Job]:
    """64 independent capsule-in-shear cases: cubic edges from {32..96}, sphere or oblate
    (c/a=0.5) capsules of radius 0.2*edge, level 3 or 4, Ca log-uniform in CA_RANGE,
    k_b/k_s0 in [0, 0.05], mass ratio drawn in [0, 2] and floored by membrane_mass_floor,
    tau~U(0.6,1), walls +-0.01."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(njobs):
        e = int(rng.choice(BATCH_EDGES))
        level = 3 if rng.uniform() < 0.5 else 4
        jobs.append(_shear_job(rng, (e, e, e), level, storage, steps, f"batch{seed}_{j}", j))
    return jobs


SERVE_LATTICES = ((48, 48, 48), (64, 64, 64), (96, 48, 96), (128, 64, 128))
SETTLING_EDGES = (48, 64, 80)


def abraham_terminal_velocity(d: float, gravity: float, density_ratio: float, nu: float) -> float:
    """Terminal settling speed of a sphere of diameter d from Abraham's drag law (Sec. 2,
    settling sphere): C_d = C_0 (1 + delta_0/sqrt(Re))^2 with C_0 delta_0^2 = 24, delta_0 = 9.06,
    u = sqrt(4 g d (gamma - 1) / (3 C_d)), Re = d u / nu; the fixed point in u is found by
    bisection.  Used only to bound run lengths of generated settling jobs."""
    delta0 = 9.06
    c0 = 24.0 / delta0 ** 2

    def excess(u):
        re = max(d * u / nu, 1e-300)
        cd = c0 * (1.0 + delta0 / math.sqrt(re)) ** 2
        return u - math.sqrt(4.0 * gravity * d * (density_ratio - 1.0) / (3.0 * cd))

    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if excess(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    return hi


def _settle_job(rng: np.random.Generator, edge: int, storage: int, steps: int, name: str,
                tag: int) -> Job:
    """Rigid sphere settling in the paper's box proportions (Sec. 2, settling sphere):
    L_x = L_y = 6.67 d, L_z = 10.67 d, released at rest 8 d above the floor, tau = 0.7,
    gravity 1e-5 along -z, level-4 sphere (mean edge 0.27..0.45 lattice units for these sizes,
    about the 0.3..0.5 Lagrangian/Eulerian spacing ratio the paper recommends).  The run length
    is cut so that, moving at the unbounded terminal speed (an upper bound inside the box), the
    sphere stops at least one diameter above the floor."""
    d = edge / 6.67
    nz = int(round(10.67 * d))
    ratio = float(rng.choice(SETTLING_DENSITY_RATIOS))
    tau, g = 0.7, 1e-5
    lat = LatticeSpec(edge, edge, nz, tau, storage=storage, **closed_box())
    body = BodySpec(rigid=1, ks0=0.0, kb=0.0, kv=0.0, mass_ratio=ratio, gravity=(0.0, 0.0, -g))
    z0 = 8.0 * d - 0.5
    xyz, tri = spheroid_mesh(4, (0.5 * d,) * 3, ((edge - 1) / 2.0, (edge - 1) / 2.0, z0))
    u_inf = abraham_terminal_velocity(d, g, ratio, (tau - 0.5) / 3.0)
    steps = int(min(steps, (z0 - 1.5 * d) / u_inf))
    return Job(name, lat, body, xyz, tri, steps, tag=tag, kind="settling")


def serving_stream(seed: int = 0, rate_per_s: float = 4.0, window_s: float = 1800.0,
                   storage: int = STORE_F16, steps_range=(2000, 10000),
                   levels=(3, 4, 5), lattices=SERVE_LATTICES,
                   max_jobs: Optional[int] = None) -> List[Job]:
    """Poisson arrivals of capsule-shear and settling jobs (50/50), run lengths uniform in
    steps_range.  Shear jobs take the batching parameters on lattices drawn from 48^3 ..
    128x64x128 with mesh levels from {3,4,5} (642-10242 nodes); settling jobs are built by
    _settle_job on square-section boxes of edge 48..80 (at most 80x80x128 nodes)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs: List[Job] = []
    while True:
        t += float(rng.exponential(1.0 / rate_per_s))
        if t > window_s or (max_jobs is not None and len(jobs) >= max_jobs):
            break
        dims = tuple(int(v) for v in lattices[int(rng.integers(len(lattices)))])
        level = int(levels[int(rng.integers(len(levels)))])
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        tag = len(jobs)
        if rng.uniform() < 0.5:
            job = _shear_job(rng, dims, level, storage, steps, f"serve{seed}_{tag}", tag)
        else:
            edge = int(SETTLING_EDGES[int(rng.integers(len(SETTLING_EDGES)))])
            job = _settle_job(rng, edge, storage, steps, f"serve{seed}_{tag}", tag)
        job.arrival_s = t
        jobs.append(job)
    return jobs


# ---------------------------------------------------------------- fields


def random_fields(shape: Tuple[int, int, int], seed: int, amp_rho: float = 1e-3,
                  amp_u: float = 1e-2) -> Tuple[np.ndarray, np.ndarray]:
    """Smooth random density and velocity fields on an (nx, ny, nz) lattice for initial
    conditions of parity runs: rho = 1 + amp_rho*noise, u = amp_u*noise, built from a few
    random Fourier modes so that every axis is periodic.  Layout: rho[N], u[3][N] with node
    index x + nx*(y + ny*z)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def field():
        acc = np.zeros((nz, ny, nx))
        for _ in range(4):
            kx, ky, kz = (int(v) for v in rng.integers(0, 3, size=3))
            ph = rng.uniform(0, 2 * np.pi)
            acc += rng.standard_normal() * np.cos(
                2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
        return acc / 4.0

    rho = 1.0 + amp_rho * field()
    u = np.stack([amp_u * field() for _ in range(3)])
    return rho.reshape(-1).copy(), u.reshape(3, -1).copy()


def random_populations(n: int, seed: int) -> np.ndarray:
    """Arbitrary (non-equilibrium) population values f[19][n] in (0.01, 0.1) for
    permutation tests of pure streaming."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.01, 0.1, size=(19, n))
