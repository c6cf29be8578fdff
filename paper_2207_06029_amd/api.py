"""Python face of liblbib: thin wrappers with the C ABI's names (include/lbib.h).  They only
convert arguments; the time stepping, immersed boundary and structure updates all run in the
library's HIP kernels on the GPU."""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L


def _stream_handle(stream) -> Optional[int]:
    """Accept None, an int hipStream_t, or a torch.cuda.Stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def lattice_desc(spec, storage: Optional[int] = None) -> L.lbib_lattice_desc:
    d = L.lbib_lattice_desc()
    d.nx, d.ny, d.nz = int(spec.nx), int(spec.ny), int(spec.nz)
    d.storage = int(spec.storage if storage is None else storage)
    d.tau = float(spec.tau)
    for f in range(6):
        d.bc[f] = int(spec.bc[f])
        for a in range(3):
            d.wall_u[f][a] = float(spec.wall_u[f][a])
    for a in range(3):
        d.body_force[a] = float(spec.body_force[a])
    return d


def body_desc(spec) -> L.lbib_body_desc:
    d = L.lbib_body_desc()
    d.rigid = int(spec.rigid)
    d.integrator = int(getattr(spec, "integrator", 0))
    d.ks0, d.thickness, d.kb, d.kv = float(spec.ks0), float(spec.thickness), float(spec.kb), float(spec.kv)
    d.mass_ratio = float(spec.mass_ratio)
    for a in range(3):
        d.gravity[a] = float(spec.gravity[a])
    d.mls_rw, d.mls_alpha = float(spec.mls_rw), float(spec.mls_alpha)
    d.probe_len, d.shell_h = float(spec.probe_len), float(spec.shell_h)
    return d


def workspace_bytes(spec, max_nv: int = 0, max_nt: int = 0) -> int:
    out = ctypes.c_size_t()
    d = lattice_desc(spec)
    L.check(L.load().lbib_workspace_bytes(ctypes.byref(d), max_nv, max_nt, ctypes.byref(out)))
    return out.value


class Lattice:
    """lbib_lattice: one lattice with its bodies.  `spec` has the fields of lbib_lattice_desc."""

    def __init__(self, spec=None, stream=None, workspace_ptr: int = 0, workspace_bytes: int = 0,
                 _handle=None, _owner=True):
        self._lib = L.load()
        if _handle is not None:
            self._h = _handle
        else:
            h = ctypes.c_void_p()
            d = lattice_desc(spec)
            L.check(self._lib.lbib_lattice_create(ctypes.byref(d), _stream_handle(stream),
                                                  workspace_ptr or None, workspace_bytes,
                                                  ctypes.byref(h)))
            self._h = h
            self.nx, self.ny, self.nz = int(spec.nx), int(spec.ny), int(spec.nz)
        self._owner = _owner

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def destroy(self):
        if getattr(self, "_h", None) and self._owner:
            self._lib.lbib_lattice_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    # fluid
    def init(self, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        L.check(self._lib.lbib_lattice_init(self._h, None if r is None else L.dptr(r),
                                            None if v is None else L.dptr(v)))

    def step(self, n: int = 1):
        L.check(self._lib.lbib_step(self._h, int(n)))

    def stream_only(self, n: int = 1):
        L.check(self._lib.lbib_stream_only(self._h, int(n)))

    def sync(self):
        L.check(self._lib.lbib_sync(self._h))

    @property
    def step_count(self) -> int:
        return int(self._lib.lbib_step_count(self._h))

    def macros(self):
        rho = np.zeros(self.n)
        u = np.zeros(3 * self.n)
        L.check(self._lib.lbib_get_macros(self._h, L.dptr(rho), L.dptr(u)))
        return rho, u.reshape(3, self.n)

    def macros_noalloc(self, rho: Optional[np.ndarray] = None, u: Optional[np.ndarray] = None):
        """lbib_get_macros_noalloc into caller arrays (float64, N and 3N; None skips a field)."""
        for a, m in ((rho, 1), (u, 3)):
            if a is not None and (a.dtype != np.float64 or a.size != m * self.n or not a.flags.c_contiguous):
                raise ValueError("outputs must be C-contiguous float64 arrays of N and 3N entries")
        L.check(self._lib.lbib_get_macros_noalloc(self._h, None if rho is None else L.dptr(rho),
                                                  None if u is None else L.dptr(u)))
        return rho, u

    def populations(self):
        f = np.zeros(19 * self.n)
        L.check(self._lib.lbib_get_populations(self._h, L.dptr(f)))
        return f.reshape(19, self.n)

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        L.check(self._lib.lbib_set_populations(self._h, L.dptr(f)))

    # bodies
    def add_body(self, spec, xyz, tri) -> int:
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1)
        tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1)
        d = body_desc(spec)
        bid = ctypes.c_int32()
        L.check(self._lib.lbib_body_add(self._h, ctypes.byref(d), L.dptr(xyz), len(xyz) // 3,
                                        L.iptr(tri), len(tri) // 3, ctypes.byref(bid)))
        return bid.value

    def counts(self, b: int):
        nv, nt = ctypes.c_int32(), ctypes.c_int32()
        L.check(self._lib.lbib_body_count(self._h, b, ctypes.byref(nv), ctypes.byref(nt)))
        return nv.value, nt.value

    def set_velocity(self, b: int, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        L.check(self._lib.lbib_body_set_velocity(self._h, b, L.dptr(v)))

    def body_state(self, b: int):
        nv, _ = self.counts(b)
        x = np.zeros(3 * nv)
        v = np.zeros(3 * nv)
        L.check(self._lib.lbib_body_get_state(self._h, b, L.dptr(x), L.dptr(v)))
        return x.reshape(nv, 3), v.reshape(nv, 3)

    def body_forces(self, b: int):
        nv, _ = self.counts(b)
        fv = np.zeros(3 * nv)
        F = np.zeros(3)
        M = np.zeros(3)
        L.check(self._lib.lbib_body_get_forces(self._h, b, L.dptr(fv), L.dptr(F), L.dptr(M)))
        return fv.reshape(nv, 3), F, M

    # timing
    def set_timing(self, enable=True):
        """enable: False / 0 off; True / 1 every sweep launch; n > 1 every n-th launch."""
        L.check(self._lib.lbib_set_timing(self._h, int(enable)))

    def kernel_time(self, kernel: int = 0):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        L.check(self._lib.lbib_kernel_time(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value


def _job_struct(job, storage: int, keep: list) -> L.lbib_job:
    s = L.lbib_job()
    s.lattice = lattice_desc(job.lattice, storage)
    if job.body is not None and job.xyz is not None:
        s.body = body_desc(job.body)
        xyz = np.ascontiguousarray(job.xyz, dtype=np.float64).reshape(-1)
        tri = np.ascontiguousarray(job.tri, dtype=np.int32).reshape(-1)
        keep += [xyz, tri]
        s.xyz = L.dptr(xyz)
        s.tri = L.iptr(tri)
        s.nv = len(xyz) // 3
        s.nt = len(tri) // 3
    s.steps = int(job.steps)
    s.tag = int(job.tag)
    return s


class Batch:
    """lbib_batch: many lattices advanced by shared launches."""

    def __init__(self, jobs: Sequence, storage: int = 0, autotune: bool = False,
                 tune_cache: Optional[str] = None, use_graph: bool = False, stream=None):
        self._lib = L.load()
        keep: list = []
        arr = (L.lbib_job * len(jobs))(*[_job_struct(j, storage, keep) for j in jobs])
        opts = L.lbib_batch_opts()
        opts.storage = int(storage)
        opts.autotune = int(bool(autotune))
        opts.tune_cache = tune_cache.encode() if tune_cache else None
        opts.use_graph = int(bool(use_graph))
        h = ctypes.c_void_p()
        L.check(self._lib.lbib_batch_create(arr, len(jobs), ctypes.byref(opts),
                                            _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.jobs = list(jobs)

    def destroy(self):
        if getattr(self, "_h", None):
            self._lib.lbib_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def step(self, n: int = 1):
        L.check(self._lib.lbib_batch_step(self._h, int(n)))

    def sync(self):
        L.check(self._lib.lbib_batch_sync(self._h))

    def lattice(self, j: int) -> Lattice:
        h = ctypes.c_void_p()
        L.check(self._lib.lbib_batch_lattice(self._h, int(j), ctypes.byref(h)))
        lat = Lattice(_handle=h, _owner=False)
        spec = self.jobs[j].lattice
        lat.nx, lat.ny, lat.nz = int(spec.nx), int(spec.ny), int(spec.nz)
        lat._batch_ref = self
        return lat

    def launch_shape(self):
        b, n = ctypes.c_int32(), ctypes.c_int32()
        L.check(self._lib.lbib_batch_launch_shape(self._h, ctypes.byref(b), ctypes.byref(n)))
        return b.value, n.value


class Server:
    """lbib_server: continuous batching over slots sized once for the memory budget; jobs are
    spliced into free slots and retired in place."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, steps_per_tick: int,
                 storage: int = 1, use_graph: bool = False, stream=None, dry_run: bool = False,
                 slot_nodes: int = 0, slot_vertices: int = 0, slot_triangles: int = 0):
        self._lib = L.load()
        o = L.lbib_server_opts()
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.max_slots = int(max_slots)
        o.steps_per_tick = int(steps_per_tick)
        o.storage = int(storage)
        o.use_graph = int(bool(use_graph))
        o.dry_run = int(bool(dry_run))
        o.slot_nodes = int(slot_nodes)
        o.slot_vertices = int(slot_vertices)
        o.slot_triangles = int(slot_triangles)
        h = ctypes.c_void_p()
        L.check(self._lib.lbib_server_create(ctypes.byref(o), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.storage = storage
        self._nv = {}

    def destroy(self):
        if getattr(self, "_h", None):
            self._lib.lbib_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def submit(self, job) -> int:
        keep: list = []
        s = _job_struct(job, self.storage, keep)
        jid = ctypes.c_uint64()
        L.check(self._lib.lbib_server_submit(self._h, ctypes.byref(s), ctypes.byref(jid)))
        self._nv[jid.value] = int(s.nv)
        return jid.value

    def tick(self):
        L.check(self._lib.lbib_server_tick(self._h))

    def poll(self, cap: int = 64, with_positions: bool = False) -> List[dict]:
        res = (L.lbib_result * cap)()
        bufs = []
        if with_positions:
            # one buffer large enough for the biggest queued mesh
            nvmax = max(self._nv.values()) if self._nv else 0
            for i in range(cap):
                b = np.zeros(3 * max(nvmax, 1))
                bufs.append(b)
                res[i].xyz = L.dptr(b)
        n = ctypes.c_int32()
        L.check(self._lib.lbib_server_poll(self._h, res, cap, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            r = res[i]
            d = dict(id=r.id, tag=r.tag, status=r.status, nv=r.nv, steps_done=r.steps_done,
                     t_submit_ns=r.t_submit_ns, t_admit_ns=r.t_admit_ns, t_finish_ns=r.t_finish_ns,
                     F=np.array(r.F[:]), M=np.array(r.M[:]))
            if with_positions:
                d["xyz"] = bufs[i][:3 * r.nv].reshape(-1, 3).copy()
            out.append(d)
        return out

    def stats(self):
        q, r = ctypes.c_int32(), ctypes.c_int32()
        b = ctypes.c_uint64()
        nu = ctypes.c_double()
        L.check(self._lib.lbib_server_stats(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b), ctypes.byref(nu)))
        return dict(queued=q.value, resident=r.value, resident_bytes=b.value, node_updates=nu.value)

    def info(self):
        s = ctypes.c_int32()
        sb, db = ctypes.c_uint64(), ctypes.c_uint64()
        L.check(self._lib.lbib_server_info(self._h, ctypes.byref(s), ctypes.byref(sb), ctypes.byref(db)))
        return dict(slots=s.value, slot_bytes=sb.value, device_bytes=db.value)
