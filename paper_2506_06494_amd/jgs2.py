"""Thin ctypes binding of libjgs2 (see include/jgs2.h for every contract).

Argument marshalling only: every step of the solve runs in the HIP library.
Raises if the library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjgs2.so")
BOUNDS_LIB_PATH = os.path.join(HERE, "libjgs2_bounds.so")  # index-checked sweep kernels

OK, E_INVALID, E_OOM, E_HIP, E_NOT_READY, E_DIVERGED, E_INFEASIBLE, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
E_BOUNDS = -8
NOT_CONVERGED = 1
PLAIN, CUBATURE, DAMPER, EXACT = 0, 3, 4, 5
JACOBI, GS = 0, 1
MAX_PLANES = 8

STATUS_NAMES = {1: "NOT_CONVERGED", 0: "OK", -1: "INVALID", -2: "OOM", -3: "HIP", -4: "NOT_READY", -5: "DIVERGED",
                -6: "INFEASIBLE", -7: "NONFINITE", -8: "BOUNDS"}


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_double * 3), ("variant", C.c_int32), ("order", C.c_int32),
                ("omega", C.c_double), ("rel_tol", C.c_double), ("max_sweeps", C.c_int32),
                ("check_every", C.c_int32), ("d_hat", C.c_double), ("kappa", C.c_double),
                ("n_planes", C.c_int32), ("line_search", C.c_int32), ("planes", (C.c_double * 4) * MAX_PLANES),
                ("adj_rel_tol", C.c_double), ("adj_max_sweeps", C.c_int32), ("use_graph", C.c_int32),
                ("exact_drop", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("status", C.c_int32), ("r0", C.c_double), ("r_final", C.c_double),
                ("seconds", C.c_double), ("ls_halvings", C.c_int32), ("reserved", C.c_int32),
                ("dx_norm", C.c_double)]


class AdjointStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("status", C.c_int32), ("adjoint_sweeps", C.c_int64),
                ("forward_sweeps", C.c_int64), ("max_rel_res", C.c_double), ("seconds", C.c_double)]


EXPORTS = ["jgs2_default_params", "jgs2_create", "jgs2_destroy", "jgs2_last_error", "jgs2_set_params",
           "jgs2_set_stream", "jgs2_upload_mesh", "jgs2_set_material", "jgs2_precompute",
           "jgs2_import_correction", "jgs2_export_correction", "jgs2_get_ring_sizes", "jgs2_get_poses",
           "jgs2_set_state", "jgs2_get_state", "jgs2_step", "jgs2_begin_step", "jgs2_iterate", "jgs2_end_step",
           "jgs2_residual", "jgs2_energy", "jgs2_get_phase1", "jgs2_get_coloring", "jgs2_set_profiling",
           "jgs2_kernel_times", "jgs2_rollout", "jgs2_rollout_backward", "jgs2_set_bodies", "jgs2_get_body_stats",
           "jgs2_set_tuning", "jgs2_get_tuning", "jgs2_autotune", "jgs2_set_streaming", "jgs2_set_material_log_e",
           "jgs2_energy_noalloc", "jgs2_set_state_device", "jgs2_get_state_device", "jgs2_exact_tiles", "jgs2_set_persistent", "jgs2_precompute_cached",
           "jgs2_bounds_report", "jgs2_bounds_selftest", "jgs2_exact_tiles_fp16"]

KERNELS = ["phase1", "phase2", "plain", "commit", "reduce", "predict", "velocity", "energy", "linear", "paramgrad",
           "adjvec", "damper", "rot", "exact", "hvec", "symv", "ysum"]

_lib = None


def load(path: str = LIB_PATH):
    """Loads libjgs2 (no GPU needed to load)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2506_06494_amd.build.build() first")
    lib = C.CDLL(path)
    P = C.POINTER
    d, i32, u8 = P(C.c_double), P(C.c_int32), P(C.c_uint8)
    sig = {
        "jgs2_default_params": (None, [P(Params)]),
        "jgs2_create": (C.c_int32, [P(Params), P(C.c_void_p)]),
        "jgs2_destroy": (None, [C.c_void_p]),
        "jgs2_last_error": (C.c_char_p, [C.c_void_p]),
        "jgs2_set_params": (C.c_int32, [C.c_void_p, P(Params)]),
        "jgs2_set_stream": (C.c_int32, [C.c_void_p, C.c_void_p]),
        "jgs2_upload_mesh": (C.c_int32, [C.c_void_p, C.c_int32, d, C.c_int32, i32, u8]),
        "jgs2_set_material": (C.c_int32, [C.c_void_p, d, d, d]),
        "jgs2_set_material_log_e": (C.c_int32, [C.c_void_p, d, d, d]),
        "jgs2_precompute": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_uint64]),
        "jgs2_import_correction": (C.c_int32, [C.c_void_p, C.c_int32, d, i32, d, d]),
        "jgs2_export_correction": (C.c_int32, [C.c_void_p, C.c_int32, d, i32, d, d, d]),
        "jgs2_get_ring_sizes": (C.c_int32, [C.c_void_p, i32, i32]),
        "jgs2_get_poses": (C.c_int32, [C.c_void_p, i32, d]),
        "jgs2_exact_tiles": (C.c_int32, [C.c_void_p, P(C.c_int64), P(C.c_int64), d, d]),
        "jgs2_set_persistent": (C.c_int32, [C.c_void_p, C.c_int32]),
        "jgs2_bounds_report": (C.c_int32, [C.c_void_p, P(C.c_int32), P(C.c_int64), P(C.c_int64), C.c_int32]),
        "jgs2_bounds_selftest": (C.c_int32, [C.c_void_p]),
        "jgs2_exact_tiles_fp16": (C.c_int32, [C.c_void_p]),
        "jgs2_precompute_cached": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_uint64, C.c_char_p,
                                               P(C.c_int32)]),
        "jgs2_set_state": (C.c_int32, [C.c_void_p, d, d]),
        "jgs2_get_state": (C.c_int32, [C.c_void_p, d, d]),
        "jgs2_set_state_device": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
        "jgs2_get_state_device": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
        "jgs2_step": (C.c_int32, [C.c_void_p, P(StepStats)]),
        "jgs2_begin_step": (C.c_int32, [C.c_void_p]),
        "jgs2_iterate": (C.c_int32, [C.c_void_p, C.c_int32, d]),
        "jgs2_end_step": (C.c_int32, [C.c_void_p]),
        "jgs2_residual": (C.c_int32, [C.c_void_p, d, d]),
        "jgs2_energy": (C.c_int32, [C.c_void_p, d]),
        "jgs2_energy_noalloc": (C.c_int32, [C.c_void_p, d]),
        "jgs2_get_phase1": (C.c_int32, [C.c_void_p, d, d]),
        "jgs2_get_coloring": (C.c_int32, [C.c_void_p, i32, i32]),
        "jgs2_set_profiling": (C.c_int32, [C.c_void_p, C.c_int32]),
        "jgs2_kernel_times": (C.c_int32, [C.c_void_p, d, P(C.c_int64)]),
        "jgs2_rollout": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, P(StepStats)]),
        "jgs2_rollout_backward": (C.c_int32, [C.c_void_p, d, d, d, d, d, d, P(AdjointStats)]),
        "jgs2_set_bodies": (C.c_int32, [C.c_void_p, C.c_int32, i32]),
        "jgs2_get_body_stats": (C.c_int32, [C.c_void_p, i32, i32, d]),
        "jgs2_set_tuning": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32]),
        "jgs2_get_tuning": (C.c_int32, [C.c_void_p, i32, i32]),
        "jgs2_set_streaming": (C.c_int32, [C.c_void_p, C.c_int32]),
        "jgs2_autotune": (C.c_int32, [C.c_void_p, C.c_int32, i32, i32, d]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


_hip = None


def device_synchronize():
    """hipDeviceSynchronize in the HIP runtime libjgs2 is linked against (the
    system ROCm one; a torch build may carry a runtime of its own, which does
    not see work queued through this one)."""
    global _hip
    load()
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so.7")
        _hip.hipDeviceSynchronize.restype = C.c_int
    r = _hip.hipDeviceSynchronize()
    if r != 0:
        raise JGS2Error(E_HIP, f"hipDeviceSynchronize returned {r}")


class JGS2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def default_params() -> Params:
    p = Params()
    load().jgs2_default_params(C.byref(p))
    return p


def make_params(**kw) -> Params:
    p = default_params()
    planes = kw.pop("planes", None)
    for k, v in kw.items():
        if k == "gravity":
            for i in range(3):
                p.gravity[i] = float(v[i])
        else:
            setattr(p, k, v)
    if planes is not None:
        planes = np.asarray(planes, dtype=np.float64).reshape(-1, 4)
        p.n_planes = planes.shape[0]
        for i in range(planes.shape[0]):
            for k in range(4):
                p.planes[i][k] = float(planes[i, k])
    return p


class Solver:
    """One libjgs2 handle."""

    def __init__(self, params: Params | None = None, **kw):
        self.lib = load()
        self.params = params if params is not None else make_params(**kw)
        h = C.c_void_p()
        r = self.lib.jgs2_create(C.byref(self.params), C.byref(h))
        if r != OK:
            raise JGS2Error(r, "jgs2_create failed (no gfx950 device?)")
        self.h = h
        self.nV = self.nT = 0

    def _chk(self, r):
        """Raises on a failure code; NOT_CONVERGED (a completed call whose
        solve stopped at its sweep cap) is returned, not raised."""
        if r < OK:
            raise JGS2Error(r, self.lib.jgs2_last_error(self.h).decode())
        return r

    def close(self):
        if getattr(self, "h", None):
            self.lib.jgs2_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **kw):
        for k, v in kw.items():
            if k == "gravity":
                for i in range(3):
                    self.params.gravity[i] = float(v[i])
            else:
                setattr(self.params, k, v)
        self._chk(self.lib.jgs2_set_params(self.h, C.byref(self.params)))

    def set_stream(self, stream_handle: int):
        self._chk(self.lib.jgs2_set_stream(self.h, C.c_void_p(stream_handle)))

    def upload_mesh(self, X, tets, pinned):
        X = np.ascontiguousarray(X, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        pinned = np.ascontiguousarray(pinned, dtype=np.uint8)
        self.nV, self.nT = X.shape[0], tets.shape[0]
        self.X, self.pinned = X.copy(), pinned.astype(bool)
        self._chk(self.lib.jgs2_upload_mesh(self.h, self.nV, _dptr(X), self.nT, _iptr(tets),
                                            pinned.ctypes.data_as(C.POINTER(C.c_uint8))))

    def set_material(self, E, nu, rho):
        arr = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (self.nT,))) for a in (E, nu, rho)]
        self._chk(self.lib.jgs2_set_material(self.h, *[_dptr(a) for a in arr]))

    def set_material_log_e(self, log_E, nu, rho):
        """Per-tet E = exp(log_E), taken inside the library."""
        arr = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (self.nT,)))
               for a in (log_E, nu, rho)]
        self._chk(self.lib.jgs2_set_material_log_e(self.h, *[_dptr(a) for a in arr]))

    def precompute(self, samples=4, n_cand=64, seed=0, cache=None):
        """GPU precompute; with `cache` (a file path) load it from there when
        the file matches these inputs, else compute and write it.  Returns
        True when loaded from the cache."""
        if cache is None:
            self._chk(self.lib.jgs2_precompute(self.h, samples, n_cand, C.c_uint64(seed)))
            return False
        loaded = C.c_int32()
        self._chk(self.lib.jgs2_precompute_cached(self.h, samples, n_cand, C.c_uint64(seed),
                                                  os.fsencode(cache), C.byref(loaded)))
        return bool(loaded.value)

    def ring_sizes(self):
        n = C.c_int32()
        self._chk(self.lib.jgs2_get_ring_sizes(self.h, C.byref(n), None))
        sizes = np.zeros(n.value, dtype=np.int32)
        self._chk(self.lib.jgs2_get_ring_sizes(self.h, C.byref(n), _iptr(sizes)))
        return sizes

    def poses(self):
        n = C.c_int32()
        ev = np.zeros(32)
        self._chk(self.lib.jgs2_get_poses(self.h, C.byref(n), _dptr(ev)))
        return ev[:n.value].copy()

    def import_correction(self, S, U_ring, samples, weights, U_samp):
        U_ring = np.ascontiguousarray(U_ring, dtype=np.float64)
        samples = np.ascontiguousarray(samples, dtype=np.int32)
        weights = np.ascontiguousarray(weights, dtype=np.float64)
        U_samp = np.ascontiguousarray(U_samp, dtype=np.float64)
        self._chk(self.lib.jgs2_import_correction(self.h, S, _dptr(U_ring), _iptr(samples), _dptr(weights),
                                                  _dptr(U_samp)))

    def export_correction(self, S):
        sizes = self.ring_sizes()
        nf = sizes.size
        U_ring = np.zeros((int(sizes.sum()), 3, 3))
        samples = np.zeros((nf, S), dtype=np.int32)
        weights = np.zeros((nf, S))
        U_samp = np.zeros((nf, S, 4, 3, 3))
        fit = np.zeros(nf)
        self._chk(self.lib.jgs2_export_correction(self.h, S, _dptr(U_ring), _iptr(samples), _dptr(weights),
                                                  _dptr(U_samp), _dptr(fit)))
        return dict(sizes=sizes, U_ring=U_ring, samples=samples, weights=weights, U_samp=U_samp, fit=fit)

    def set_state(self, x, v):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        self._chk(self.lib.jgs2_set_state(self.h, _dptr(x), _dptr(v)))

    def get_state(self):
        x = np.zeros((self.nV, 3))
        v = np.zeros((self.nV, 3))
        self._chk(self.lib.jgs2_get_state(self.h, _dptr(x), _dptr(v)))
        return x, v

    def step(self, raise_on_error=True):
        st = StepStats()
        r = self.lib.jgs2_step(self.h, C.byref(st))
        if raise_on_error:
            self._chk(r)
        return dict(status=r, sweeps=st.sweeps, r0=st.r0, r_final=st.r_final, seconds=st.seconds,
                    ls_halvings=st.ls_halvings, dx_norm=st.dx_norm)

    def begin_step(self):
        self._chk(self.lib.jgs2_begin_step(self.h))

    def iterate(self, n, raise_on_error=True):
        rel = C.c_double()
        r = self.lib.jgs2_iterate(self.h, int(n), C.byref(rel))
        if raise_on_error:
            self._chk(r)
        return rel.value

    def end_step(self):
        self._chk(self.lib.jgs2_end_step(self.h))

    def residual(self):
        a, r = C.c_double(), C.c_double()
        self._chk(self.lib.jgs2_residual(self.h, C.byref(a), C.byref(r)))
        return a.value, r.value

    def set_bodies(self, body_of_vertex):
        b = np.ascontiguousarray(body_of_vertex, dtype=np.int32)
        self.n_bodies = int(b.max()) + 1
        self._chk(self.lib.jgs2_set_bodies(self.h, self.n_bodies, _iptr(b)))

    def body_stats(self):
        """(sweeps per body, |g_b| / |g_b(x0)| per body) at the last check."""
        n = C.c_int32()
        self._chk(self.lib.jgs2_get_body_stats(self.h, C.byref(n), None, None))
        sw = np.zeros(n.value, dtype=np.int32)
        rel = np.zeros(n.value)
        self._chk(self.lib.jgs2_get_body_stats(self.h, C.byref(n), _iptr(sw), _dptr(rel)))
        return sw, rel

    def set_tuning(self, lanes_per_vertex, block):
        self._chk(self.lib.jgs2_set_tuning(self.h, int(lanes_per_vertex), int(block)))

    def set_streaming(self, mode):
        """-1 auto, 0 cached, 1 streamed incidence records (cache hint only)."""
        self._chk(self.lib.jgs2_set_streaming(self.h, int(mode)))

    def tuning(self):
        a, b = C.c_int32(), C.c_int32()
        self._chk(self.lib.jgs2_get_tuning(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self, sweeps=16):
        """Times every launch shape; keeps and returns the fastest
        (lanes_per_vertex, block) and the 4 x 4 table of times (ms)."""
        a, b = C.c_int32(), C.c_int32()
        ms = np.zeros(16)
        self._chk(self.lib.jgs2_autotune(self.h, int(sweeps), C.byref(a), C.byref(b), _dptr(ms)))
        return (a.value, b.value), ms.reshape(4, 4)

    def rollout(self, n_steps, ckpt_every=5):
        """n_steps forward steps from the current state, keeping device
        checkpoints every ckpt_every steps; returns the last step's stats."""
        st = StepStats()
        r = self._chk(self.lib.jgs2_rollout(self.h, int(n_steps), int(ckpt_every), C.byref(st)))
        return dict(status=r, sweeps=st.sweeps, r0=st.r0, r_final=st.r_final, seconds=st.seconds)

    def rollout_backward(self, xbar, vbar=None):
        """Pulls (xbar_N, vbar_N) back through the last rollout; returns
        (thetabar (nT,), xbar_0, vbar_0, stats); stats["ubar"] is the
        cotangent of one initial velocity shared by the free vertices."""
        xbar = np.ascontiguousarray(xbar, dtype=np.float64).reshape(self.nV, 3)
        vb = None if vbar is None else np.ascontiguousarray(vbar, dtype=np.float64).reshape(self.nV, 3)
        th = np.zeros(self.nT)
        xb0 = np.zeros((self.nV, 3))
        vb0 = np.zeros((self.nV, 3))
        ub = np.zeros(3)
        st = AdjointStats()
        r = self._chk(self.lib.jgs2_rollout_backward(self.h, _dptr(xbar), None if vb is None else _dptr(vb),
                                                     _dptr(th), _dptr(xb0), _dptr(vb0), _dptr(ub), C.byref(st)))
        return th, xb0, vb0, dict(status=r, steps=st.steps, adjoint_sweeps=st.adjoint_sweeps,
                                  forward_sweeps=st.forward_sweeps, max_rel_res=st.max_rel_res,
                                  seconds=st.seconds, ubar=ub)

    def bounds_report(self, clear=False):
        """Bounds-checked build only: the first failed index check as
        (kernel source line, index, extent); line 0 when none failed."""
        line, idx, ext = C.c_int32(), C.c_int64(), C.c_int64()
        self._chk(self.lib.jgs2_bounds_report(self.h, C.byref(line), C.byref(idx), C.byref(ext), int(clear)))
        return line.value, idx.value, ext.value

    def bounds_selftest(self):
        self._chk(self.lib.jgs2_bounds_selftest(self.h))

    def set_persistent(self, on=True):
        """Coloured GS groups of the plain variant as one cooperative launch."""
        self._chk(self.lib.jgs2_set_persistent(self.h, int(on)))

    def exact_tiles(self):
        """Stored H-bar^-1 tiles of the exact variant, those the sweep streams
        under exact_drop, their bytes and the partial-sum bytes a sweep writes."""
        nt, nl, b, pb = C.c_int64(), C.c_int64(), C.c_double(), C.c_double()
        self._chk(self.lib.jgs2_exact_tiles(self.h, C.byref(nt), C.byref(nl), C.byref(b), C.byref(pb)))
        return dict(n_tiles=nt.value, n_live=nl.value, live_bytes=b.value, part_bytes=pb.value)

    def exact_tiles_fp16(self):
        """H-bar^-1 tiles stored in FP16 (scaled per tile) from here on."""
        self._chk(self.lib.jgs2_exact_tiles_fp16(self.h))

    def set_state_device(self, d_x, d_v):
        """d_x, d_v: device addresses (ints) of nV x 3 doubles."""
        self._chk(self.lib.jgs2_set_state_device(self.h, C.c_void_p(d_x), C.c_void_p(d_v)))

    def get_state_device(self, d_x, d_v):
        self._chk(self.lib.jgs2_get_state_device(self.h, C.c_void_p(d_x), C.c_void_p(d_v)))

    def energy(self):
        e = C.c_double()
        self._chk(self.lib.jgs2_energy(self.h, C.byref(e)))
        return e.value

    def energy_noalloc(self):
        """jgs2_energy_noalloc: the same energy with the library's static
        device scratch instead of handle-owned buffers."""
        e = C.c_double()
        self._chk(self.lib.jgs2_energy_noalloc(self.h, C.byref(e)))
        return e.value

    def phase1(self):
        g = np.zeros((self.nV, 3))
        R = np.zeros((self.nV, 3, 3))
        self._chk(self.lib.jgs2_get_phase1(self.h, _dptr(g), _dptr(R)))
        return g, R

    def set_profiling(self, on=True):
        self._chk(self.lib.jgs2_set_profiling(self.h, 1 if on else 0))

    def kernel_times(self):
        """{kernel name: (total ms, launches)} since profiling was enabled."""
        ms = np.zeros(len(KERNELS))
        n = np.zeros(len(KERNELS), dtype=np.int64)
        self._chk(self.lib.jgs2_kernel_times(self.h, _dptr(ms), n.ctypes.data_as(C.POINTER(C.c_int64))))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}

    def coloring(self):
        c = np.zeros(self.nV, dtype=np.int32)
        n = C.c_int32()
        self._chk(self.lib.jgs2_get_coloring(self.h, _iptr(c), C.byref(n)))
        return c, n.value
