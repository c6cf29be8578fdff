"""FP64 CPU oracle of the D3Q19 BGK lattice-Boltzmann / dynamic immersed-boundary scheme.

TEST INFRASTRUCTURE ONLY.  The oracle is a plain C implementation of the scheme in
arXiv 2207.06029 Sec. 1, used to check the GPU implementation.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the GPU product path never
does.  It shares no code with the GPU path.

Arguments that describe a lattice or a body are duck-typed (any object with the attribute
names below), so this package imports nothing from the GPU package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbib_oracle.c")
_SO = os.path.join(_HERE, "liblbib_oracle.so")

OK, EINVAL, ENOMEM, EUNSTABLE, EDOMAIN = 0, -1, -2, -4, -7


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
                               "-Wno-unused-parameter", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def build_variant(replacements, out_dir: str, name: str = "variant") -> str:
    """Compile a copy of the oracle with textual replacements [(old, new), ...] applied (each
    old text must occur exactly once) into out_dir; for tests that plant a mistake in the
    oracle and check that a pin catches it.  Returns the library path."""
    src = open(_SRC).read()
    for old, new in replacements:
        if src.count(old) != 1:
            raise ValueError(f"replacement target found {src.count(old)} times: {old!r}")
        src = src.replace(old, new)
    os.makedirs(out_dir, exist_ok=True)
    c = os.path.join(out_dir, name + ".c")
    so = os.path.join(out_dir, "lib" + name + ".so")
    with open(c, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                           "-ffp-contract=off", "-w", "-I", _HERE, "-o", so, c, "-lm"])
    return so


class use_library:
    """Context manager: route the module's calls (and lattices created inside) to another
    build of the oracle, e.g. one from build_variant."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        lib()
        self.saved = _lib
        L = ctypes.CDLL(self.path)
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_step_count.restype = ctypes.c_int64
        L.orc_lattice_create.argtypes = [ctypes.POINTER(_LatticeDesc), ctypes.POINTER(ctypes.c_void_p)]
        L.orc_lattice_destroy.argtypes = [ctypes.c_void_p]
        _lib = L
        return L

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


class _LatticeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("tau", ctypes.c_double),
                ("bc", ctypes.c_int32 * 6), ("wall_u", (ctypes.c_double * 3) * 6),
                ("body_force", ctypes.c_double * 3)]


class _BodyDesc(ctypes.Structure):
    _fields_ = [("rigid", ctypes.c_int32), ("integrator", ctypes.c_int32),
                ("ks0", ctypes.c_double), ("thickness", ctypes.c_double),
                ("kb", ctypes.c_double), ("kv", ctypes.c_double),
                ("mass_ratio", ctypes.c_double), ("gravity", ctypes.c_double * 3),
                ("mls_rw", ctypes.c_double), ("mls_alpha", ctypes.c_double),
                ("probe_len", ctypes.c_double), ("shell_h", ctypes.c_double)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_step_count.restype = ctypes.c_int64
        L.orc_lattice_create.argtypes = [ctypes.POINTER(_LatticeDesc), ctypes.POINTER(ctypes.c_void_p)]
        for name in ("orc_lattice_destroy",):
            getattr(L, name).argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


def _p(a: np.ndarray, ty=_D):
    return a.ctypes.data_as(ty)


def _check(rc: int):
    if rc != OK:
        raise OracleError(rc, lib().orc_last_error().decode())


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def d3q19():
    e = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    lib().orc_d3q19(_p(e, _I32), _p(w))
    return e.reshape(19, 3), w


def equilibrium(rho: float, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    lib().orc_equilibrium(ctypes.c_double(rho), _p(u), _p(out))
    return out


def guo_forcing(tau: float, u, F) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    lib().orc_guo_forcing(ctypes.c_double(tau), _p(u), _p(F), _p(out))
    return out


def collide_node(tau: float, f, F) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    lib().orc_collide_node(ctypes.c_double(tau), _p(f), _p(F), _p(out))
    return out


def wall_closure(axis: int, side: int, uw, F, f) -> np.ndarray:
    f = np.array(f, dtype=np.float64)
    uw = np.ascontiguousarray(uw, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    lib().orc_wall_closure(int(axis), int(side), _p(uw), _p(F), _p(f))
    return f


def corner_closure(side, rho: float, uw, F, f) -> np.ndarray:
    f = np.array(f, dtype=np.float64)
    sd = np.ascontiguousarray(side, dtype=np.int32)
    uw = np.ascontiguousarray(uw, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    rc = lib().orc_corner_closure(_p(sd, _I32), ctypes.c_double(rho), _p(uw), _p(F), _p(f))
    if rc != 0:
        raise OracleError(rc, "singular corner system")
    return f


def _lattice_desc(spec) -> _LatticeDesc:
    d = _LatticeDesc()
    d.nx, d.ny, d.nz = int(spec.nx), int(spec.ny), int(spec.nz)
    d.tau = float(spec.tau)
    for i in range(6):
        d.bc[i] = int(spec.bc[i])
        for a in range(3):
            d.wall_u[i][a] = float(spec.wall_u[i][a])
    for a in range(3):
        d.body_force[a] = float(spec.body_force[a])
    return d


def _body_desc(spec) -> _BodyDesc:
    d = _BodyDesc()
    d.rigid = int(spec.rigid)
    d.integrator = int(getattr(spec, "integrator", 0))
    d.ks0, d.thickness, d.kb, d.kv = float(spec.ks0), float(spec.thickness), float(spec.kb), float(spec.kv)
    d.mass_ratio = float(spec.mass_ratio)
    for a in range(3):
        d.gravity[a] = float(spec.gravity[a])
    d.mls_rw, d.mls_alpha = float(spec.mls_rw), float(spec.mls_alpha)
    d.probe_len, d.shell_h = float(spec.probe_len), float(spec.shell_h)
    return d


class Lattice:
    """One oracle lattice.  `spec` has nx, ny, nz, tau, bc[6], wall_u[6][3], body_force[3]."""

    def __init__(self, spec):
        self.nx, self.ny, self.nz = int(spec.nx), int(spec.ny), int(spec.nz)
        self.n = self.nx * self.ny * self.nz
        self.tau = float(spec.tau)
        self._L = lib()
        h = ctypes.c_void_p()
        d = _lattice_desc(spec)
        self._check(self._L.orc_lattice_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.bodies = []

    def _check(self, rc: int):
        if rc != OK:
            raise OracleError(rc, self._L.orc_last_error().decode())

    def close(self):
        if self._h:
            self._L.orc_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # fluid ---------------------------------------------------------------
    def init(self, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        self._check(self._L.orc_lattice_init(self._h, None if r is None else _p(r),
                                      None if v is None else _p(v)))

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        self._check(self._L.orc_set_populations(self._h, _p(f)))

    def populations(self) -> np.ndarray:
        f = np.zeros(19 * self.n)
        self._check(self._L.orc_get_populations(self._h, _p(f)))
        return f.reshape(19, self.n)

    def macros(self):
        rho = np.zeros(self.n)
        u = np.zeros(3 * self.n)
        self._check(self._L.orc_get_macros(self._h, _p(rho), _p(u)))
        return rho, u.reshape(3, self.n)

    def step(self, n: int = 1):
        self._check(self._L.orc_step(self._h, int(n)))

    def stream_only(self, n: int = 1):
        self._check(self._L.orc_stream_only(self._h, int(n)))

    @property
    def step_count(self) -> int:
        return int(self._L.orc_step_count(self._h))

    # bodies --------------------------------------------------------------
    def add_body(self, spec, xyz, tri) -> int:
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1)
        tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1)
        d = _body_desc(spec)
        bid = ctypes.c_int32()
        self._check(self._L.orc_body_add(self._h, ctypes.byref(d), _p(xyz), len(xyz) // 3,
                                  _p(tri, _I32), len(tri) // 3, ctypes.byref(bid)))
        self.bodies.append(bid.value)
        return bid.value

    def counts(self, b: int):
        nv, nt, ne = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._L.orc_body_counts(self._h, b, ctypes.byref(nv), ctypes.byref(nt), ctypes.byref(ne)))
        return nv.value, nt.value, ne.value

    def set_velocity(self, b: int, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        self._check(self._L.orc_body_set_velocity(self._h, b, _p(v)))

    def body_state(self, b: int):
        nv, _, _ = self.counts(b)
        x = np.zeros(3 * nv)
        v = np.zeros(3 * nv)
        self._check(self._L.orc_body_get_state(self._h, b, _p(x), _p(v)))
        return x.reshape(nv, 3), v.reshape(nv, 3)

    def body_forces(self, b: int):
        nv, _, _ = self.counts(b)
        fv = np.zeros(3 * nv)
        F = np.zeros(3)
        M = np.zeros(3)
        self._check(self._L.orc_body_get_forces(self._h, b, _p(fv), _p(F), _p(M)))
        return fv.reshape(nv, 3), F, M

    def topology(self, b: int):
        _, _, ne = self.counts(b)
        e = np.zeros(2 * ne, dtype=np.int32)
        h = np.zeros(4 * ne, dtype=np.int32)
        self._check(self._L.orc_body_topology(self._h, b, _p(e, _I32), _p(h, _I32)))
        return e.reshape(ne, 2), h.reshape(ne, 4)

    def rest(self, b: int):
        nv, nt, ne = self.counts(b)
        l0, ks, th0 = np.zeros(ne), np.zeros(ne), np.zeros(ne)
        A0 = np.zeros(nt)
        sc = np.zeros(4)
        self._check(self._L.orc_body_rest(self._h, b, _p(l0), _p(ks), _p(th0), _p(A0), _p(sc)))
        return dict(l0=l0, ks=ks, theta0=th0, A0=A0, V0=sc[0], S0=sc[1], mv=sc[2], mass=sc[3])

    def set_positions(self, b: int, xyz):
        """Membrane at rest at xyz (x^n = x^{n-1} = xyz, vertex velocities 0)."""
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1)
        self._check(self._L.orc_body_set_positions(self._h, b, _p(x)))

    def rigid_state(self, b: int):
        """Centre X, rotation R (x = X + R x_body), velocity u and angular velocity omega."""
        X, R, u, om = np.zeros(3), np.zeros(9), np.zeros(3), np.zeros(3)
        self._check(self._L.orc_body_rigid_state(self._h, b, _p(X), _p(R), _p(u), _p(om)))
        return X, R.reshape(3, 3), u, om

    def rigid_advance(self, b: int, F, M):
        """The rigid part of the structure update with hydrodynamic totals F, M given."""
        F = np.ascontiguousarray(F, dtype=np.float64)
        M = np.ascontiguousarray(M, dtype=np.float64)
        self._check(self._L.orc_rigid_advance(self._h, b, _p(F), _p(M)))

    def rigid_props(self, b: int):
        X0 = np.zeros(3)
        m = ctypes.c_double()
        I = np.zeros(9)
        self._check(self._L.orc_body_rigid_props(self._h, b, _p(X0), ctypes.byref(m), _p(I)))
        return X0, m.value, I.reshape(3, 3)

    def membrane_forces(self, b: int, xyz=None):
        nv, _, _ = self.counts(b)
        F = np.zeros(3 * nv)
        E = np.zeros(3)
        x = None if xyz is None else np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1)
        self._check(self._L.orc_membrane_forces(self._h, b, None if x is None else _p(x), _p(F), _p(E)))
        return F.reshape(nv, 3), E

    def mls(self, x, rw: float = 1.3, alpha: float = 0.3):
        x = np.ascontiguousarray(x, dtype=np.float64)
        idx = np.zeros(27, dtype=np.int64)
        d = np.zeros(81)
        phi = np.zeros(27)
        g = np.zeros(81)
        c = ctypes.c_int32()
        self._check(self._L.orc_mls(self._h, _p(x), ctypes.c_double(rw), ctypes.c_double(alpha),
                             _p(idx, _I64), _p(d), _p(phi), _p(g), ctypes.byref(c)))
        k = c.value
        return idx[:k].copy(), d[:3 * k].reshape(k, 3).copy(), phi[:k].copy(), g[:3 * k].reshape(k, 3).copy()

    def ib_force(self):
        nt_total = sum(self.counts(b)[1] for b in self.bodies)
        flb = np.zeros(3 * self.n)
        U = np.zeros(3 * max(nt_total, 1))
        Fl = np.zeros(3 * max(nt_total, 1))
        self._check(self._L.orc_ib_force(self._h, _p(flb), _p(U), _p(Fl)))
        return flb.reshape(3, self.n), U[:3 * nt_total].reshape(-1, 3), Fl[:3 * nt_total].reshape(-1, 3)

    def probe_forces(self, b: int):
        _, nt, _ = self.counts(b)
        F = np.zeros(3 * nt)
        self._check(self._L.orc_body_probe_forces(self._h, b, _p(F)))
        return F.reshape(nt, 3)
