"""GPU parity of the lattice part (Sec. 1.1) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from paper_2207_06029_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2207_06029_amd import api as A
    return A


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _roll(f0, e, k, shape):
    nx, ny, nz = shape
    out = np.empty_like(f0)
    for i in range(19):
        g = f0[i].reshape(nz, ny, nx)
        out[i] = np.roll(g, shift=(k * e[i, 2], k * e[i, 1], k * e[i, 0]), axis=(0, 1, 2)).reshape(-1)
    return out


@pytest.mark.parametrize("storage", [I.STORE_F32, I.STORE_F16, I.STORE_BF16])
def test_streaming_is_bitwise_permutation(api, orc, storage):
    shape = (37, 5, 3)   # a ragged tail in every launch shape
    spec = I.LatticeSpec(*shape, 0.8, storage=storage)
    lat = api.Lattice(spec)
    lat.set_populations(I.random_populations(spec.n, seed=1))
    f0 = lat.populations()
    e, _ = orc.d3q19()
    lat.stream_only(9)
    f = lat.populations()
    np.testing.assert_array_equal(f, _roll(f0, e, 9, shape))


def test_streaming_with_resting_bounceback_walls_matches_oracle_bitwise(api, orc):
    spec = I.LatticeSpec(6, 7, 9, 0.8, **I.closed_box())
    lat = api.Lattice(spec)
    lat.set_populations(I.random_populations(spec.n, seed=2))
    f0 = lat.populations()
    ref = orc.Lattice(spec)
    ref.set_populations(f0)
    lat.stream_only(5)
    ref.stream_only(5)
    np.testing.assert_array_equal(lat.populations(), ref.populations())


def test_set_get_roundtrip(api, orc):
    spec = I.LatticeSpec(11, 6, 5, 0.8)
    lat = api.Lattice(spec)
    _, w = orc.d3q19()
    f = I.random_populations(spec.n, seed=3)
    lat.set_populations(f)
    g = lat.populations()
    # stored as FP32 deviations from the weights: error at most half an FP32 ulp of |f - w|
    dev = np.abs(f - w[:, None]).astype(np.float32)
    bound = 0.5 * np.spacing(dev).astype(np.float64) * (1 + 1e-6)
    assert (np.abs(g - f) <= bound).all()


def _fluid_case(spec, seed, steps, orc, api, amp_u=1e-2):
    rho, u = I.random_fields((spec.nx, spec.ny, spec.nz), seed=seed, amp_u=amp_u)
    lat = api.Lattice(spec)
    lat.init(rho, u)
    ref = orc.Lattice(spec)
    ref.init(rho, u)
    lat.step(steps)
    lat.sync()
    ref.step(steps)
    return lat.macros(), ref.macros(), lat, ref


@pytest.mark.parametrize("steps", [1, 60])
def test_collide_stream_periodic_with_body_force(api, orc, steps):
    spec = I.LatticeSpec(23, 12, 9, 0.8, body_force=(2e-6, -1e-6, 5e-7))
    (rho, u), (rr, ur), lat, ref = _fluid_case(spec, 4, steps, orc, api)
    assert rel_l2(u, ur) < 2e-6
    assert np.abs(rho - rr).max() < 1e-7
    f, fr = lat.populations(), ref.populations()
    assert np.abs(f - fr).max() < 2e-8


def test_zouhe_shear_walls_parity(api, orc):
    spec = I.LatticeSpec(9, 17, 6, 0.7, **I.shear_walls(0.02))
    (rho, u), (rr, ur), *_ = _fluid_case(spec, 5, 200, orc, api)
    assert rel_l2(u, ur) < 2e-6
    assert np.abs(rho - rr).max() < 1e-7


def test_zouhe_body_force_poiseuille_matches_closed_form(api):
    ny = 17
    g = 1e-6
    tau = 0.8
    nu = (tau - 0.5) / 3
    spec = I.LatticeSpec(4, ny, 3, tau, bc=(0, 0, 1, 1, 0, 0), body_force=(g, 0.0, 0.0))
    lat = api.Lattice(spec)
    lat.step(20000)
    rho, u = lat.macros()
    y = np.tile(np.repeat(np.arange(ny), 4), 3)
    exact = g / (2 * nu) * y * (ny - 1 - y)
    ug = u[0] + g / (2 * rho)
    assert np.abs(ug - exact).max() < 1e-4 * exact.max()


def test_moving_bounceback_box_parity(api, orc):
    wall_u = ((0, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0), (0.01, -0.005, 0.0), (-0.01, 0.0, 0.0))
    spec = I.LatticeSpec(10, 8, 13, 0.9, bc=(2,) * 6, wall_u=wall_u)
    (rho, u), (rr, ur), *_ = _fluid_case(spec, 6, 150, orc, api)
    assert rel_l2(u, ur) < 2e-6
    assert np.abs(rho - rr).max() < 1e-7


def _reduced_precision_error(api, orc, storage):
    spec = I.LatticeSpec(16, 17, 8, 0.8, storage=storage, **I.shear_walls(0.02))
    (rho, u), (rr, ur), *_ = _fluid_case(spec, 7, 300, orc, api)
    err = rel_l2(u, ur)
    print(f"storage {storage}: rel-L2 u* after 300 steps {err:.3e}")
    return err


def test_reduced_precision_storage_fp16(api, orc):
    """FP16 shifted deviations meet the 1e-3 reduced-precision gate."""
    assert _reduced_precision_error(api, orc, I.STORE_F16) < 1e-3


@pytest.mark.xfail(strict=True, reason="BF16 storage does not meet the 1e-3 reduced-precision gate: "
                   "its 8 significand bits give about 2e-2 on this case")
def test_reduced_precision_storage_bf16_gate(api, orc):
    assert _reduced_precision_error(api, orc, I.STORE_BF16) < 1e-3


def test_errors_surface(api):
    spec = I.LatticeSpec(8, 8, 8, 0.8)
    lat = api.Lattice(spec)
    with pytest.raises(api.L.LbibError) as ei:
        lat.body_state(3)
    assert ei.value.code == -6
    # invalid timing requests are rejected; a sampling period times every n-th sweep launch
    with pytest.raises(api.L.LbibError) as ei:
        lat.set_timing(-1)
    assert ei.value.code == -1
    with pytest.raises(api.L.LbibError) as ei:
        lat.kernel_time(2)
    assert ei.value.code == -1
    lat.set_timing(4)
    lat.step(10)
    ms, n = lat.kernel_time(0)
    assert n == 3 and ms > 0.0           # launches 0, 4 and 8 of the 10
    ms, n = lat.kernel_time(1)
    assert n == 10
    lat.set_timing(0)
    # an unknown vertex-update mode is refused at upload
    xyz, tri = I.spheroid_mesh(1, (2.0, 2.0, 2.0), (3.5, 3.5, 3.5))
    with pytest.raises(api.L.LbibError) as ei:
        lat.add_body(I.BodySpec(rigid=0, ks0=0.01, kb=0.0, kv=0.0, mass_ratio=1.0, integrator=3), xyz, tri)
    assert ei.value.code == -1
