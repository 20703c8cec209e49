"""Python binding of the UGKWP C ABI (include/ugkwp.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libugkwp.so.  PyTorch provides the
device workspace (one uint8 tensor) and the stream.  There is no fallback: if the library
or a GPU is missing, construction fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libugkwp.so")

OK, E_ARG, E_MESH, E_CAPACITY, E_LOST, E_NONPHYS, E_DEVICE, E_STATE = range(8)
STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_MESH", 3: "E_CAPACITY", 4: "E_LOST", 5: "E_NONPHYS",
                6: "E_DEVICE", 7: "E_STATE"}

# every entry point the header declares
SYMBOLS = ("ugkwp_workspace_bytes", "ugkwp_init_mesh", "ugkwp_init_state", "ugkwp_step", "ugkwp_moments",
           "ugkwp_particle_count", "ugkwp_export_particles", "ugkwp_geometry", "ugkwp_profile_enable",
           "ugkwp_profile_read", "ugkwp_profile_slot_name", "ugkwp_last_error", "ugkwp_destroy",
           "ugkwp_instance_stats", "ugkwp_instance_cells", "ugkwp_graph_enable", "ugkwp_set_launch",
           "ugkwp_get_launch", "ugkwp_autotune", "ugkwp_autotune_cached", "ugkwp_profile_mask",
           "ugkwp_set_averaging", "ugkwp_average", "ugkwp_export_state", "ugkwp_import_state", "ugkwp_init_mesh_static", "ugkwp_static_workspace_bytes")
N_PROFILE_SLOTS = 12


class UgkwpBC(C.Structure):
    _fields_ = [("type", C.c_int32), ("T_w", C.c_double), ("U_w", C.c_double * 3), ("W_inf", C.c_double * 5),
                ("shift", C.c_double * 3)]


class UgkwpMesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.POINTER(C.c_double)), ("n_cells", C.c_int64),
                ("cell_type", C.POINTER(C.c_uint8)), ("cell_node_off", C.POINTER(C.c_int64)),
                ("cell_nodes", C.POINTER(C.c_int64)), ("n_bfaces", C.c_int64),
                ("bface_nodes", C.POINTER(C.c_int64)), ("bface_bc", C.POINTER(C.c_int32)),
                ("n_bc", C.c_int32), ("bc", C.POINTER(UgkwpBC))]


class UgkwpParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mu_ref", C.c_double), ("omega", C.c_double), ("cfl", C.c_double),
                ("c2", C.c_double), ("n_ref", C.c_int32), ("n_min", C.c_int32), ("recon", C.c_int32),
                ("precision", C.c_int32), ("capacity", C.c_int64), ("max_crossings", C.c_int32),
                ("seed", C.c_uint64), ("venkat_k", C.c_double), ("sampling", C.c_int32),
                ("gks_steps", C.c_int32), ("prandtl", C.c_double)]


class UgkwpStats(C.Structure):
    _fields_ = [("dt", C.c_double), ("t", C.c_double), ("step", C.c_int64), ("n_alive", C.c_int64),
                ("n_sampled", C.c_int64), ("n_collided", C.c_int64), ("n_escaped", C.c_int64),
                ("n_moved", C.c_int64), ("crossings", C.c_int64), ("wall_hits", C.c_int64),
                ("error_word", C.c_uint32), ("moved_total", C.c_int64), ("n_injected", C.c_int64),
                ("max_crossings_seen", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class UgkwpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libugkwp.so (built by __graft_entry__.build() / paper_2007_13091_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        P, vp = C.POINTER, C.c_void_p
        L.ugkwp_workspace_bytes.restype = C.c_int32
        L.ugkwp_workspace_bytes.argtypes = [P(UgkwpMesh), C.c_int32, P(UgkwpParams), P(C.c_size_t)]
        L.ugkwp_init_mesh.restype = C.c_int32
        L.ugkwp_init_mesh.argtypes = [P(vp), P(UgkwpMesh), C.c_int32, P(UgkwpParams), vp, C.c_size_t, vp]
        L.ugkwp_init_mesh_static.restype = C.c_int32
        L.ugkwp_init_mesh_static.argtypes = [P(vp), P(UgkwpMesh), C.c_int32, P(UgkwpParams), vp]
        L.ugkwp_static_workspace_bytes.restype = C.c_size_t
        L.ugkwp_static_workspace_bytes.argtypes = []
        L.ugkwp_instance_stats.restype = C.c_int32
        L.ugkwp_instance_stats.argtypes = [vp, C.c_int32, P(UgkwpStats)]
        L.ugkwp_profile_mask.restype = C.c_int32
        L.ugkwp_profile_mask.argtypes = [vp, C.c_uint32]
        L.ugkwp_graph_enable.restype = C.c_int32
        L.ugkwp_graph_enable.argtypes = [vp, C.c_int32]
        L.ugkwp_set_launch.restype = C.c_int32
        L.ugkwp_set_launch.argtypes = [vp, P(C.c_int32)]
        L.ugkwp_get_launch.restype = C.c_int32
        L.ugkwp_get_launch.argtypes = [vp, P(C.c_int32)]
        L.ugkwp_autotune.restype = C.c_int32
        L.ugkwp_autotune.argtypes = [vp, C.c_int32, P(C.c_int32)]
        L.ugkwp_autotune_cached.restype = C.c_int32
        L.ugkwp_autotune_cached.argtypes = [vp, C.c_int32, C.c_char_p, P(C.c_int32), P(C.c_int32)]
        L.ugkwp_instance_cells.restype = C.c_int32
        L.ugkwp_instance_cells.argtypes = [vp, C.c_int32, P(C.c_int64), P(C.c_int64)]
        L.ugkwp_init_state.restype = C.c_int32
        L.ugkwp_init_state.argtypes = [vp, P(C.c_double)]
        L.ugkwp_step.restype = C.c_int32
        L.ugkwp_step.argtypes = [vp, C.c_int32, P(UgkwpStats)]
        L.ugkwp_moments.restype = C.c_int32
        L.ugkwp_moments.argtypes = [vp, C.c_int32, vp, C.c_int32]
        L.ugkwp_set_averaging.restype = C.c_int32
        L.ugkwp_set_averaging.argtypes = [vp, C.c_int64]
        L.ugkwp_average.restype = C.c_int32
        L.ugkwp_average.argtypes = [vp, vp, C.c_int32, P(C.c_double), P(C.c_int64)]
        L.ugkwp_particle_count.restype = C.c_int32
        L.ugkwp_particle_count.argtypes = [vp, P(C.c_int64)]
        L.ugkwp_export_particles.restype = C.c_int32
        L.ugkwp_export_particles.argtypes = [vp, P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_int32),
                                             P(C.c_uint64), P(C.c_double)]
        L.ugkwp_export_state.restype = C.c_int32
        L.ugkwp_export_state.argtypes = [vp, P(C.c_double), P(C.c_double), P(C.c_int64), P(C.c_double)]
        L.ugkwp_import_state.restype = C.c_int32
        L.ugkwp_import_state.argtypes = [vp, P(C.c_double), P(C.c_double), C.c_int64, P(C.c_double),
                                         P(C.c_double), P(C.c_double), P(C.c_int32), P(C.c_uint64),
                                         P(C.c_double), P(C.c_int64), P(C.c_double)]
        L.ugkwp_geometry.restype = C.c_int32
        L.ugkwp_geometry.argtypes = [vp, P(C.c_double), P(C.c_double), P(C.c_double)]
        L.ugkwp_profile_enable.restype = C.c_int32
        L.ugkwp_profile_enable.argtypes = [vp, C.c_int32]
        L.ugkwp_profile_read.restype = C.c_int32
        L.ugkwp_profile_read.argtypes = [vp, C.c_int32, P(C.c_double), P(C.c_int64)]
        L.ugkwp_profile_slot_name.restype = C.c_char_p
        L.ugkwp_profile_slot_name.argtypes = [C.c_int32]
        L.ugkwp_last_error.restype = C.c_char_p
        L.ugkwp_last_error.argtypes = [vp]
        L.ugkwp_destroy.restype = None
        L.ugkwp_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class _MeshArgs:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, mesh):
        self.xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
        self.ct = np.ascontiguousarray(mesh.cell_type, dtype=np.uint8)
        self.off = np.ascontiguousarray(mesh.cell_node_off, dtype=np.int64)
        self.cn = np.ascontiguousarray(mesh.cell_nodes, dtype=np.int64)
        self.bf = np.ascontiguousarray(mesh.bface_nodes, dtype=np.int64).reshape(-1, 4)
        self.bt = np.ascontiguousarray(mesh.bface_bc, dtype=np.int32)
        self.bcs = (UgkwpBC * max(len(mesh.bcs), 1))()
        for i, b in enumerate(mesh.bcs):
            self.bcs[i].type = b.type
            self.bcs[i].T_w = b.Tw
            for d in range(3):
                self.bcs[i].U_w[d] = b.Uw[d]
            for k in range(5):
                self.bcs[i].W_inf[k] = b.Winf[k]
            for d in range(3):
                self.bcs[i].shift[d] = getattr(b, "shift", (0.0, 0.0, 0.0))[d]
        self.s = UgkwpMesh(self.xyz.shape[0], _ptr(self.xyz, C.c_double), self.ct.shape[0], _ptr(self.ct, C.c_uint8),
                           _ptr(self.off, C.c_int64), _ptr(self.cn, C.c_int64), self.bf.shape[0],
                           _ptr(self.bf, C.c_int64), _ptr(self.bt, C.c_int32), len(mesh.bcs), self.bcs)


def make_params(p, capacity=0, precision=0) -> UgkwpParams:
    return UgkwpParams(p.gamma, p.mu_ref, p.omega, p.cfl, p.c2, p.n_ref, p.n_min, int(getattr(p, "recon", 0)),
                       precision, capacity, p.max_crossings, p.seed, float(getattr(p, "venkat_k", 1.0)),
                       int(getattr(p, "sampling", 0)), int(getattr(p, "gks_steps", 0)),
                       float(getattr(p, "prandtl", 1.0)))


class _BatchArgs:
    """C arrays of meshes and parameters for n instances (single objects count as one)."""

    def __init__(self, meshes, params, capacity=0, precision=0):
        if not isinstance(meshes, (list, tuple)):
            meshes, params = [meshes], [params]
        if not isinstance(params, (list, tuple)):
            params = [params] * len(meshes)
        if len(params) != len(meshes):
            raise ValueError("one params per mesh")
        caps = capacity if isinstance(capacity, (list, tuple)) else [capacity] * len(meshes)
        self.n = len(meshes)
        self.margs = [_MeshArgs(m) for m in meshes]
        self.m = (UgkwpMesh * self.n)(*[a.s for a in self.margs])
        self.p = (UgkwpParams * self.n)(*[make_params(pp, cc, precision=precision) for pp, cc in zip(params, caps)])
        self.ncells = [m.n_cells for m in meshes]


def workspace_bytes(mesh, params, capacity=0, precision=0) -> int:
    """Device bytes the library needs (host-side computation: mesh checks and layout).
    mesh/params may be lists (a batch of instances)."""
    L = lib()
    b = _BatchArgs(mesh, params, capacity, precision)
    n = C.c_size_t(0)
    st = L.ugkwp_workspace_bytes(b.m, b.n, b.p, C.byref(n))
    if st != OK:
        raise UgkwpError(st, L.ugkwp_last_error(None).decode())
    return int(n.value)


class Solver:
    """One mesh, or a batch of independent instances (lists of meshes and params), on one
    GPU.  `mesh`, `params`: see paper_2007_13091_amd.workloads.  stream: a torch stream to
    order the work on (default: the current stream).  static_workspace: use the library's
    own static workspace (ugkwp_init_mesh_static; nothing is allocated, small meshes only,
    one such solver per GPU at a time)."""

    def __init__(self, mesh, params, capacity=0, precision=0, device="cuda", stream=None, static_workspace=False):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a GPU (the HIP library has no CPU path)")
        L = lib()
        self.torch = torch
        b = _BatchArgs(mesh, params, capacity, precision)
        self.n_inst = b.n
        self.nc = int(sum(b.ncells))
        n = C.c_size_t(0)
        st = L.ugkwp_workspace_bytes(b.m, b.n, b.p, C.byref(n))
        if st != OK:
            raise UgkwpError(st, L.ugkwp_last_error(None).decode())
        self.precision = precision
        h = C.c_void_p(0)
        if static_workspace:
            self.ws = None
            self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
            st = L.ugkwp_init_mesh_static(C.byref(h), b.m, b.n, b.p, C.c_void_p(self.stream.cuda_stream))
        else:
            self.ws = torch.empty(int(n.value), dtype=torch.uint8, device=device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
            st = L.ugkwp_init_mesh(C.byref(h), b.m, b.n, b.p, C.c_void_p(self.ws.data_ptr()), n.value,
                                   C.c_void_p(self.stream.cuda_stream))
        if st != OK:
            raise UgkwpError(st, L.ugkwp_last_error(None).decode())
        self.h = h

    def _check(self, st):
        if st != OK:
            raise UgkwpError(st, lib().ugkwp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().ugkwp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_state(self, W0):
        W0 = np.ascontiguousarray(W0, dtype=np.float64).reshape(self.nc, 5)
        self._check(lib().ugkwp_init_state(self.h, _ptr(W0, C.c_double)))

    def step(self, n=1, stats=True):
        """Advance n steps; returns the last step's statistics (synchronising) if stats."""
        if stats:
            s = UgkwpStats()
            self._check(lib().ugkwp_step(self.h, int(n), C.byref(s)))
            return s.as_dict()
        self._check(lib().ugkwp_step(self.h, int(n), None))
        return None

    def instance_stats(self, k):
        s = UgkwpStats()
        self._check(lib().ugkwp_instance_stats(self.h, int(k), C.byref(s)))
        return s.as_dict()

    def instance_cells(self, k):
        a, b = C.c_int64(0), C.c_int64(0)
        self._check(lib().ugkwp_instance_cells(self.h, int(k), C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def graph(self, on=True):
        """Replay each step from a captured hip graph (needs a created stream)."""
        self._check(lib().ugkwp_graph_enable(self.h, 1 if on else 0))

    def launch_config(self, cfg=None):
        """Get (and with cfg, first set) the launch shapes (stream_bs, stream_ilp, sample_wpb, flux_bs)."""
        if cfg is not None:
            a = np.ascontiguousarray(cfg, dtype=np.int32)
            self._check(lib().ugkwp_set_launch(self.h, _ptr(a, C.c_int32)))
        out = np.zeros(4, dtype=np.int32)
        self._check(lib().ugkwp_get_launch(self.h, _ptr(out, C.c_int32)))
        return tuple(int(v) for v in out)

    def autotune(self, steps_per_trial=3, cache=None):
        """Pick the fastest launch shapes on real steps (the state advances).  cache: the path
        of a result cache (JSON lines); a hit sets the cached shapes without stepping.  Returns
        the shapes, and with a cache also whether it was a hit."""
        out = np.zeros(4, dtype=np.int32)
        if cache is None:
            self._check(lib().ugkwp_autotune(self.h, int(steps_per_trial), _ptr(out, C.c_int32)))
            return tuple(int(v) for v in out)
        hit = C.c_int32(0)
        self._check(lib().ugkwp_autotune_cached(self.h, int(steps_per_trial), str(cache).encode(),
                                                _ptr(out, C.c_int32), C.byref(hit)))
        return tuple(int(v) for v in out), bool(hit.value)

    def moments(self, which=0):
        out = np.zeros((self.nc, 5), dtype=np.float64)
        self._check(lib().ugkwp_moments(self.h, int(which), C.c_void_p(out.ctypes.data), 0))
        return out

    def set_averaging(self, n_avg):
        """Time-average the steps n > n_avg from now on (Sec. 2.4(c)); n_avg < 0: off."""
        self._check(lib().ugkwp_set_averaging(self.h, int(n_avg)))

    def average(self):
        """(Wbar [n_cells][5], relative change of the last averaged step per instance, steps
        averaged per instance)."""
        out = np.zeros((self.nc, 5), dtype=np.float64)
        res = np.zeros(self.n_inst)
        n = np.zeros(self.n_inst, dtype=np.int64)
        self._check(lib().ugkwp_average(self.h, C.c_void_p(out.ctypes.data), 0, _ptr(res, C.c_double),
                                        _ptr(n, C.c_int64)))
        return out, res, n

    def particle_count(self):
        n = C.c_int64(0)
        self._check(lib().ugkwp_particle_count(self.h, C.byref(n)))
        return int(n.value)

    def particles(self):
        n = self.particle_count()
        x = np.zeros((n, 3)); u = np.zeros((n, 3)); m = np.zeros(n)
        c = np.zeros(n, dtype=np.int32); uid = np.zeros(n, dtype=np.uint64); e = np.zeros(n)
        self._check(lib().ugkwp_export_particles(self.h, _ptr(x, C.c_double), _ptr(u, C.c_double),
                                                 _ptr(m, C.c_double), _ptr(c, C.c_int32), _ptr(uid, C.c_uint64),
                                                 _ptr(e, C.c_double)))
        return dict(x=x, u=u, m=m, cell=c, uid=uid, e=e)

    def export_state(self):
        """The state between steps: W, P ([n_cells][5]; W^p = P / Omega), the particles (grouped
        by cell) and each instance's step and time."""
        W = np.zeros((self.nc, 5)); P = np.zeros((self.nc, 5))
        step = np.zeros(self.n_inst, dtype=np.int64); t = np.zeros(self.n_inst)
        self._check(lib().ugkwp_export_state(self.h, _ptr(W, C.c_double), _ptr(P, C.c_double),
                                             _ptr(step, C.c_int64), _ptr(t, C.c_double)))
        return dict(W=W, P=P, particles=self.particles(), step=step, t=t)

    def import_state(self, state):
        """Replace the state by one of export_state's (or any state of that form)."""
        W = np.ascontiguousarray(state["W"], dtype=np.float64).reshape(self.nc, 5)
        P = np.ascontiguousarray(state["P"], dtype=np.float64).reshape(self.nc, 5)
        p = state["particles"]
        n = int(np.asarray(p["uid"]).shape[0])
        x = np.ascontiguousarray(p["x"], dtype=np.float64).reshape(n, 3)
        u = np.ascontiguousarray(p["u"], dtype=np.float64).reshape(n, 3)
        m = np.ascontiguousarray(p["m"], dtype=np.float64).reshape(n)
        c = np.ascontiguousarray(p["cell"], dtype=np.int32).reshape(n)
        uid = np.ascontiguousarray(p["uid"], dtype=np.uint64).reshape(n)
        e = np.ascontiguousarray(p["e"] if p.get("e") is not None else np.zeros(n), dtype=np.float64).reshape(n)
        step = np.ascontiguousarray(np.broadcast_to(state["step"], (self.n_inst,)), dtype=np.int64)
        t = np.ascontiguousarray(np.broadcast_to(state["t"], (self.n_inst,)), dtype=np.float64)
        self._check(lib().ugkwp_import_state(self.h, _ptr(W, C.c_double), _ptr(P, C.c_double), n,
                                             _ptr(x, C.c_double), _ptr(u, C.c_double), _ptr(m, C.c_double),
                                             _ptr(c, C.c_int32), _ptr(uid, C.c_uint64), _ptr(e, C.c_double),
                                             _ptr(step, C.c_int64), _ptr(t, C.c_double)))

    def profile(self, on=True, slots=None):
        """Bracket each kernel group of a step with hip events (measurement support); slots:
        names of the groups to time (default all)."""
        if slots is None:
            mask = 0xFFFFFFFF
        else:
            names = [lib().ugkwp_profile_slot_name(k).decode() for k in range(N_PROFILE_SLOTS)]
            mask = sum(1 << names.index(n) for n in slots)
        self._check(lib().ugkwp_profile_mask(self.h, mask))
        self._check(lib().ugkwp_profile_enable(self.h, 1 if on else 0))

    def profile_read(self):
        """{slot name: (total ms, timed launches)} since the last read; waits for the stream."""
        ms = np.zeros(N_PROFILE_SLOTS)
        cnt = np.zeros(N_PROFILE_SLOTS, dtype=np.int64)
        self._check(lib().ugkwp_profile_read(self.h, N_PROFILE_SLOTS, _ptr(ms, C.c_double), _ptr(cnt, C.c_int64)))
        return {lib().ugkwp_profile_slot_name(k).decode(): (float(ms[k]), int(cnt[k])) for k in range(N_PROFILE_SLOTS)}

    def geometry(self):
        vol = np.zeros(self.nc); xc = np.zeros((self.nc, 3)); dS = np.zeros((self.nc, 3))
        self._check(lib().ugkwp_geometry(self.h, _ptr(vol, C.c_double), _ptr(xc, C.c_double), _ptr(dS, C.c_double)))
        return vol, xc, dS
