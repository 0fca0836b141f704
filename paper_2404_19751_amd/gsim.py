"""Python binding of the gsim C-ABI (``include/gsim.h``): argument marshalling
only. Every step of the hot path runs in the HIP library; if the library is
missing this module raises instead of falling back to anything else.

Arrays may be numpy arrays (host calls) or torch tensors on the GPU (the
``*_dev`` calls, which pass ``data_ptr()`` and run on the context's stream).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_libgsim.so")

OK, E_ARG, E_MESH, E_OOM, E_CAPACITY, E_DEVICE, E_STATE, E_LIMIT, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, FP32_MIXED = 0, 1
POT = {"harmonic": 0, "coulomb": 1, "gaussian": 2}
INTEG = {"overdamped": 0, "brownian": 1, "fire": 2, "verlet": 3}
PAIR_TIE, PAIR_ZERO, PAIR_GUARD = 1, 2, 4
PF_VERTEX, PF_NEAR_VERTEX, PF_CAP, PF_BOUNDARY, PF_NONFINITE = 1, 2, 4, 8, 16

EXPORTS = ["gsim_create", "gsim_destroy", "gsim_last_error", "gsim_synchronize", "gsim_mesh_upload",
           "gsim_mesh_info_get", "gsim_particles_set", "gsim_particles_get", "gsim_particles_set_dev",
           "gsim_particles_get_dev", "gsim_geodesic_pairs", "gsim_compute_forces", "gsim_displace_on_surface",
           "gsim_step", "gsim_timing_enable", "gsim_timing_get", "gsim_counters_get", "gsim_tune_set",
           "gsim_source_profile", "gsim_step_batched", "gsim_autotune", "gsim_voronoi_neighbours",
           "gsim_geodesic_pairs_dev", "gsim_compute_forces_dev", "gsim_displace_on_surface_dev",
           "gsim_particle_flags", "gsim_particle_flags_dev", "gsim_displace_on_surface_noalloc"]


class GsimError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gsim status {status}: {msg}")
        self.status = status


class MeshInfo(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nf", C.c_int32), ("n_boundary_edges", C.c_int32),
                ("n_pseudo_sources", C.c_int32), ("mean_edge", C.c_double), ("min_edge", C.c_double),
                ("max_edge", C.c_double), ("bbox_min", C.c_double * 3), ("bbox_max", C.c_double * 3)]


class PairsT(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("count", C.c_int64), ("off", C.c_void_p), ("nbr", C.c_void_p),
                ("dist", C.c_void_p), ("tan", C.c_void_p), ("flags", C.c_void_p)]


class PotentialT(C.Structure):
    _fields_ = [("kind", C.c_int32), ("k", C.c_double), ("sigma", C.c_double), ("cutoff", C.c_double)]


class IntegratorT(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dt", C.c_double), ("mobility", C.c_double), ("kT", C.c_double),
                ("friction", C.c_double), ("seed", C.c_uint64), ("max_disp", C.c_double), ("dt_max", C.c_double),
                ("alpha0", C.c_double), ("f_alpha", C.c_double), ("f_inc", C.c_double), ("f_dec", C.c_double),
                ("n_min", C.c_int32)]


class WalkStatsT(C.Structure):
    _fields_ = [("crossings", C.c_int64), ("vertex_hits", C.c_int64), ("boundary_hits", C.c_int64),
                ("cap_hits", C.c_int64), ("near_vertex", C.c_int64), ("nonfinite", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (it must have been built: ``python -m
    paper_2404_19751_amd.build`` or ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"gsim HIP library not built: {path} is missing")
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one. Loaded first, it is the runtime this library binds to as well;
    # loaded after the library has started the system runtime, it brings a
    # second runtime into the process and sees no GPU. So torch, when it is
    # installed, goes first.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    V = C.c_void_p
    sig = {
        "gsim_create": ([C.c_int, C.c_int, V, C.POINTER(V)], C.c_int),
        "gsim_destroy": ([V], None),
        "gsim_last_error": ([V], C.c_char_p),
        "gsim_synchronize": ([V], C.c_int),
        "gsim_mesh_upload": ([V, C.c_int32, V, C.c_int32, V, C.POINTER(C.c_int32)], C.c_int),
        "gsim_mesh_info_get": ([V, C.c_int32, C.POINTER(MeshInfo)], C.c_int),
        "gsim_particles_set": ([V, C.c_int32, C.c_int32, V, V, V], C.c_int),
        "gsim_particles_get": ([V, C.c_int32, V, V, V, V], C.c_int),
        "gsim_particles_set_dev": ([V, C.c_int32, C.c_int32, V, V, V], C.c_int),
        "gsim_particles_get_dev": ([V, C.c_int32, V, V, V], C.c_int),
        "gsim_geodesic_pairs": ([V, C.c_int32, C.c_double, C.POINTER(PairsT)], C.c_int),
        "gsim_geodesic_pairs_dev": ([V, C.c_int32, C.c_double, C.POINTER(PairsT)], C.c_int),
        "gsim_compute_forces": ([V, C.c_int32, C.POINTER(PotentialT), V, V], C.c_int),
        "gsim_compute_forces_dev": ([V, C.c_int32, C.POINTER(PotentialT), V, V], C.c_int),
        "gsim_displace_on_surface_dev": ([V, C.c_int32, V, C.c_int, C.POINTER(WalkStatsT)], C.c_int),
        "gsim_displace_on_surface_noalloc": ([V, C.c_int32, V, C.c_int, V, C.POINTER(WalkStatsT)], C.c_int),
        "gsim_particle_flags": ([V, C.c_int32, V], C.c_int),
        "gsim_particle_flags_dev": ([V, C.c_int32, V], C.c_int),
        "gsim_voronoi_neighbours": ([V, C.c_int32, V, V, C.c_int64, V], C.c_int),
        "gsim_displace_on_surface": ([V, C.c_int32, V, C.c_int, C.POINTER(WalkStatsT)], C.c_int),
        "gsim_step": ([V, C.c_int32, C.POINTER(PotentialT), C.POINTER(IntegratorT), C.c_int32], C.c_int),
        "gsim_timing_enable": ([V, C.c_int], C.c_int),
        "gsim_timing_get": ([V, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
        "gsim_counters_get": ([V, V], C.c_int),
        "gsim_tune_set": ([V, C.c_char_p, C.c_double], C.c_int),
        "gsim_source_profile": ([V, C.c_int, V, C.c_int32], C.c_int),
        "gsim_step_batched": ([V, C.c_int32, V, V, V, C.c_int32], C.c_int),
        "gsim_autotune": ([V, C.c_int32, V, V, V, C.c_int32, V], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _walk_stats(ws: WalkStatsT) -> dict:
    return dict(crossings=ws.crossings, vertex_hits=ws.vertex_hits, boundary_hits=ws.boundary_hits,
                cap_hits=ws.cap_hits, near_vertex=ws.near_vertex, nonfinite=ws.nonfinite)


def potential(kind="harmonic", k=1.0, sigma=1.0, cutoff=None) -> PotentialT:
    if cutoff is None:
        cutoff = sigma
    return PotentialT(POT[kind], float(k), float(sigma), float(cutoff))


def integrator(kind="overdamped", dt=0.01, mobility=1.0, kT=0.0, friction=1.0, seed=0, max_disp=0.0, dt_max=0.0,
               alpha0=0.0, f_alpha=0.0, f_inc=0.0, f_dec=0.0, n_min=0) -> IntegratorT:
    """Integrator parameters; for "fire", dt is the initial step and zero
    FIRE fields select the library defaults."""
    return IntegratorT(INTEG[kind], float(dt), float(mobility), float(kT), float(friction), int(seed), float(max_disp),
                       float(dt_max), float(alpha0), float(f_alpha), float(f_inc), float(f_dec), int(n_min))


class Context:
    """One gsim context: device buffers, stream, meshes and particle state."""

    def __init__(self, device: int = 0, precision: str = "fp64", stream=None):
        self.L = load()
        h = C.c_void_p()
        prec = FP64 if precision == "fp64" else FP32_MIXED
        sp = None
        if stream is not None:
            sp = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        st = self.L.gsim_create(int(device), prec, sp, C.byref(h))
        if st != OK:
            raise GsimError(st, "gsim_create failed")
        self.h = h
        self.precision = precision
        self._n = {}

    def close(self):
        if getattr(self, "h", None):
            self.L.gsim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != OK:
            msg = self.L.gsim_last_error(self.h)
            raise GsimError(st, msg.decode() if msg else "")

    # ---- mesh
    def mesh_upload(self, V, T) -> int:
        V = np.ascontiguousarray(V, np.float64)
        T = np.ascontiguousarray(T, np.int32)
        mid = C.c_int32()
        self._chk(self.L.gsim_mesh_upload(self.h, V.shape[0], _ptr(V), T.shape[0], _ptr(T), C.byref(mid)))
        self._n[mid.value] = 0
        return mid.value

    def mesh_info(self, mid: int) -> dict:
        mi = MeshInfo()
        self._chk(self.L.gsim_mesh_info_get(self.h, mid, C.byref(mi)))
        return dict(nv=mi.nv, nf=mi.nf, n_boundary_edges=mi.n_boundary_edges, n_pseudo_sources=mi.n_pseudo_sources,
                    mean_edge=mi.mean_edge, min_edge=mi.min_edge, max_edge=mi.max_edge)

    # ---- particles
    def particles_set(self, mid, face, bary, vel=None):
        face = np.ascontiguousarray(face, np.int32)
        bary = np.ascontiguousarray(bary, np.float64)
        v = None if vel is None else np.ascontiguousarray(vel, np.float64)
        self._chk(self.L.gsim_particles_set(self.h, mid, face.shape[0], _ptr(face), _ptr(bary), _ptr(v)))
        self._n[mid] = face.shape[0]

    def particles_set_dev(self, mid, face_t, bary_t, vel_t=None):
        self._chk(self.L.gsim_particles_set_dev(self.h, mid, int(face_t.shape[0]), _ptr(face_t), _ptr(bary_t),
                                                _ptr(vel_t)))
        self._n[mid] = int(face_t.shape[0])

    def particles_get(self, mid):
        n = self._n[mid]
        face = np.empty(n, np.int32)
        bary = np.empty((n, 3))
        vel = np.empty((n, 3))
        xyz = np.empty((n, 3))
        self._chk(self.L.gsim_particles_get(self.h, mid, _ptr(face), _ptr(bary), _ptr(vel), _ptr(xyz)))
        return face, bary, vel, xyz

    def particles_get_dev(self, mid, face_t, bary_t, vel_t=None):
        self._chk(self.L.gsim_particles_get_dev(self.h, mid, _ptr(face_t), _ptr(bary_t), _ptr(vel_t)))

    # ---- hot path
    def geodesic_pairs(self, mid, cutoff) -> dict:
        n = self._n[mid]
        off = np.empty(n + 1, np.int64)
        cap = max(16, 8 * n)
        for _ in range(2):
            nbr = np.empty(cap, np.int32)
            dist = np.empty(cap)
            tan = np.empty((cap, 3))
            flags = np.empty(cap, np.uint8)
            pt = PairsT(cap, 0, off.ctypes.data, nbr.ctypes.data, dist.ctypes.data, tan.ctypes.data,
                        flags.ctypes.data)
            st = self.L.gsim_geodesic_pairs(self.h, mid, float(cutoff), C.byref(pt))
            if st == E_CAPACITY:
                cap = int(pt.count) + 1
                continue
            self._chk(st)
            P = int(pt.count)
            return dict(off=off, nbr=nbr[:P], dist=dist[:P], tan=tan[:P], flags=flags[:P])
        raise GsimError(E_CAPACITY, "pair buffer sizing failed")

    def geodesic_pairs_dev(self, mid, cutoff, off, nbr, dist, tan, flags=None) -> int:
        """The pairs into device tensors (off[n+1] int64, nbr int32, dist
        float64, tan [cap][3] float64, flags uint8), ordered on the context's
        stream; returns the pair count (GsimError E_CAPACITY, with the count
        in its message, when the tensors are too small)."""
        pt = PairsT(int(nbr.shape[0]), 0, off.data_ptr(), nbr.data_ptr(), dist.data_ptr(), tan.data_ptr(),
                    None if flags is None else flags.data_ptr())
        self._chk(self.L.gsim_geodesic_pairs_dev(self.h, mid, float(cutoff), C.byref(pt)))
        return int(pt.count)

    def compute_forces_dev(self, mid, pot: PotentialT, force, energy=None):
        """Forces into a device tensor force[n][3] (float64) and the energy
        into energy[1] (optional), on the context's stream."""
        self._chk(self.L.gsim_compute_forces_dev(self.h, mid, C.byref(pot), _ptr(force), _ptr(energy)))

    def displace_on_surface_dev(self, mid, disp, transport_velocity=True) -> dict:
        """The shift by a device tensor disp[n][3] (float64)."""
        ws = WalkStatsT()
        self._chk(self.L.gsim_displace_on_surface_dev(self.h, mid, _ptr(disp), int(bool(transport_velocity)),
                                                      C.byref(ws)))
        return _walk_stats(ws)

    def displace_on_surface_noalloc(self, mid, disp, flags=None, transport_velocity=True) -> dict:
        """The shift by a device tensor disp[n][3] with no device allocation;
        flags (a uint8 device tensor [n], optional) receives the GSIM_PF_*
        bits."""
        ws = WalkStatsT()
        self._chk(self.L.gsim_displace_on_surface_noalloc(self.h, mid, _ptr(disp), int(bool(transport_velocity)),
                                                          _ptr(flags), C.byref(ws)))
        return _walk_stats(ws)

    def particle_flags(self, mid):
        """GSIM_PF_* bits of each particle from the last walk, step or force
        call on the mesh."""
        out = np.empty(self._n[mid], np.uint8)
        self._chk(self.L.gsim_particle_flags(self.h, mid, _ptr(out)))
        return out

    def particle_flags_dev(self, mid, out):
        self._chk(self.L.gsim_particle_flags_dev(self.h, mid, _ptr(out)))

    def compute_forces(self, mid, pot: PotentialT):
        n = self._n[mid]
        F = np.empty((n, 3))
        E = C.c_double()
        self._chk(self.L.gsim_compute_forces(self.h, mid, C.byref(pot), _ptr(F), C.c_void_p(C.addressof(E))))
        return F, E.value

    def voronoi_neighbours(self, mid):
        """In-surface Voronoi neighbours: (off[n+1], nbr) CSR, rows ascending."""
        n = self._n[mid]
        off = np.empty(n + 1, np.int64)
        cnt = C.c_int64(0)
        st = self.L.gsim_voronoi_neighbours(self.h, mid, _ptr(off), None, 0, C.byref(cnt))
        if st not in (OK, E_CAPACITY):
            self._chk(st)
        nbr = np.empty(max(cnt.value, 1), np.int32)
        self._chk(self.L.gsim_voronoi_neighbours(self.h, mid, _ptr(off), _ptr(nbr), cnt.value, C.byref(cnt)))
        return off, nbr[:cnt.value]

    def displace_on_surface(self, mid, disp, transport_velocity=True) -> dict:
        disp = np.ascontiguousarray(disp, np.float64)
        ws = WalkStatsT()
        self._chk(self.L.gsim_displace_on_surface(self.h, mid, _ptr(disp), int(bool(transport_velocity)), C.byref(ws)))
        return _walk_stats(ws)

    def step(self, mid, pot: PotentialT, integ: IntegratorT, nsteps: int = 1):
        self._chk(self.L.gsim_step(self.h, mid, C.byref(pot), C.byref(integ), int(nsteps)))

    def step_batched(self, mids, pots, integs, nsteps: int = 1):
        """nsteps steps of several surfaces in one batch (one launch per
        stage for all of them)."""
        k = len(mids)
        ids = (C.c_int32 * k)(*[int(m) for m in mids])
        pa = (PotentialT * k)(*pots)
        ia = (IntegratorT * k)(*integs)
        self._chk(self.L.gsim_step_batched(self.h, k, ids, pa, ia, int(nsteps)))

    def autotune(self, mids, pots, integs, reps: int = 3) -> dict:
        k = len(mids)
        ids = (C.c_int32 * k)(*[int(m) for m in mids])
        pa = (PotentialT * k)(*pots)
        ia = (IntegratorT * k)(*integs)
        out = np.zeros(4)
        self._chk(self.L.gsim_autotune(self.h, k, ids, pa, ia, int(reps), _ptr(out)))
        return dict(lds_stack_kb=int(out[0]), grab=int(out[1]), update_block=int(out[2]), best_ms=float(out[3]))

    def synchronize(self):
        self._chk(self.L.gsim_synchronize(self.h))

    # ---- instrumentation
    def timing(self, on: bool = True):
        self._chk(self.L.gsim_timing_enable(self.h, int(bool(on))))

    def timing_get(self, name: str):
        ms = C.c_double()
        n = C.c_int64()
        self._chk(self.L.gsim_timing_get(self.h, name.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def tune(self, **knobs):
        for k, v in knobs.items():
            self._chk(self.L.gsim_tune_set(self.h, k.encode(), float(v)))

    def source_profile_start(self):
        self._chk(self.L.gsim_source_profile(self.h, 1, None, 0))

    def source_profile_stop(self, mid):
        n = self._n[mid]
        out = np.zeros((n, 8), np.int64)
        self._chk(self.L.gsim_source_profile(self.h, 0, _ptr(out), n))
        return out

    def counters(self) -> dict:
        c = np.zeros(13, np.int64)
        self._chk(self.L.gsim_counters_get(self.h, _ptr(c)))
        return dict(windows=int(c[0]), pruned=int(c[1]), launches=int(c[2]), stale=int(c[3]), guard_sources=int(c[4]),
                    nbr_pairs=int(c[5]), limited=int(c[6]), cum_pairs=int(c[7]), cum_windows=int(c[8]),
                    cum_passes=int(c[9]), max_stack_depth=int(c[10]), nonfinite=int(c[11]),
                    crossings=int(c[12]))
