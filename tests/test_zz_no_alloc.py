"""lbib_get_macros_noalloc (the allocation-free getter, staged in the library's fixed device
array) against lbib_get_macros (staged in a buffer allocated per call), through the C ABI."""
import numpy as np
import pytest

from paper_2207_06029_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2207_06029_amd import api as A
    return A


def _both(lat):
    rho, u = lat.macros()
    r2 = np.full(lat.n, np.nan)
    u2 = np.full(3 * lat.n, np.nan)
    lat.macros_noalloc(r2, u2)
    return rho, u, r2, u2.reshape(3, lat.n)


def test_noalloc_matches_allocating_getter_on_consecutive_calls(api):
    from paper_2207_06029_amd import _lib as L
    # first call: the largest lattice the array holds (128x64x128 = LBIB_NOALLOC_MAX_NODES),
    # with a membrane driving the flow
    big = I.prolate_shear(0)
    assert big.lattice.n == L.LBIB_NOALLOC_MAX_NODES
    lat = api.Lattice(big.lattice)
    lat.add_body(big.body, big.xyz, big.tri)
    lat.init(*I.random_fields((big.lattice.nx, big.lattice.ny, big.lattice.nz), seed=5))
    lat.step(6)
    rho, u, r2, u2 = _both(lat)
    np.testing.assert_array_equal(r2, rho)
    np.testing.assert_array_equal(u2, u)
    assert np.abs(u).max() > 0
    lat.destroy()
    # second call, smaller input: the 32^3 capsule in shear, FP16 storage
    small = I.capsule_shear_small()
    spec = I.LatticeSpec(**{**small.lattice.__dict__, "storage": I.STORE_F16})
    lat2 = api.Lattice(spec)
    lat2.add_body(small.body, small.xyz, small.tri)
    lat2.step(25)
    rho, u, r2, u2 = _both(lat2)
    np.testing.assert_array_equal(r2, rho)
    np.testing.assert_array_equal(u2, u)
    # one field at a time
    r3 = np.full(lat2.n, np.nan)
    lat2.macros_noalloc(r3, None)
    np.testing.assert_array_equal(r3, rho)
    u3 = np.full(3 * lat2.n, np.nan)
    lat2.macros_noalloc(None, u3)
    np.testing.assert_array_equal(u3.reshape(3, -1), u)


def test_noalloc_follows_the_state_between_calls(api):
    spec = I.LatticeSpec(37, 5, 11, 0.8, storage=I.STORE_BF16, body_force=(1e-5, 0.0, 0.0))
    lat = api.Lattice(spec)
    lat.init(*I.random_fields((37, 5, 11), seed=9))
    for _ in range(3):
        lat.step(4)
        rho, u, r2, u2 = _both(lat)
        np.testing.assert_array_equal(r2, rho)
        np.testing.assert_array_equal(u2, u)


def test_noalloc_rejects_lattices_beyond_its_array(api):
    from paper_2207_06029_amd import _lib as L
    spec = I.LatticeSpec(129, 64, 128, 0.8, storage=I.STORE_F16)
    assert spec.n > L.LBIB_NOALLOC_MAX_NODES
    lat = api.Lattice(spec)
    rho = np.full(spec.n, 7.0)
    with pytest.raises(L.LbibError) as e:
        lat.macros_noalloc(rho, None)
    assert e.value.code == -1 and "LBIB_NOALLOC_MAX_NODES" in str(e.value)
    assert np.all(rho == 7.0)
    # the allocating getter still serves it
    r, _ = lat.macros()
    np.testing.assert_allclose(r, 1.0, atol=1e-6)
