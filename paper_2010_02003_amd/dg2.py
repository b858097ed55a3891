"""Thin Python binding of the DG2 C ABI (``include/dg2.h``, ``libdg2.so``).

Argument marshalling only: every call goes straight to the C function of the
same name without the ``dg2_`` prefix (``Sim.step`` -> ``dg2_step``), and
every step of the time integration runs in the library's HIP kernels.  There
is no fallback: if the library is not built, or no GPU is present, creating
a ``Sim`` raises.

PyTorch, when given, only supplies the HIP stream (``stream="torch"`` uses
torch's current stream so that torch events time the same queue) and device
memory (``bind_device_state``).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_void_p
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DG2_LIBRARY", os.path.join(_HERE, "libdg2.so"))

FP64, FP32 = 0, 1
NL, LL = 0, 1
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3
BC_WALL, BC_INFLOW_Q, BC_LEVEL, BC_OPEN = 0, 1, 2, 3
FLUX_HLL, FLUX_ROE = 0, 1

_STATUS = {0: "DG2_OK", -1: "DG2_EINVAL", -2: "DG2_ENOMEM", -3: "DG2_EHIP", -4: "DG2_ESTATE",
           -5: "DG2_ENUMERIC", -6: "DG2_EUNSUPPORTED"}


class DG2Error(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status
        self.message = message


class Config(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("dx", c_double), ("dy", c_double),
                ("x0", c_double), ("y0", c_double), ("prec", c_int32), ("variant", c_int32),
                ("g", c_double), ("cfl", c_double), ("tol_dry", c_double),
                ("ll_threshold", c_double), ("dt_max", c_double), ("hip_stream", c_void_p),
                ("flux", c_int32)]


# name -> (restype, argtypes)
_SIGS = {
    "dg2_config_default": (None, [POINTER(Config), c_int32, c_int32, c_double, c_double]),
    "dg2_create": (c_int32, [POINTER(Config), POINTER(c_void_p)]),
    "dg2_destroy": (None, [c_void_p]),
    "dg2_last_error": (ctypes.c_char_p, [c_void_p]),
    "dg2_set_dem_corners": (c_int32, [c_void_p, POINTER(c_double)]),
    "dg2_set_manning": (c_int32, [c_void_p, POINTER(c_double), c_double]),
    "dg2_set_initial_corners": (c_int32, [c_void_p, POINTER(c_double), c_int32, POINTER(c_double),
                                          POINTER(c_double)]),
    "dg2_set_state": (c_int32, [c_void_p, POINTER(c_double), c_double]),
    "dg2_get_state": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_int64),
                                POINTER(c_double)]),
    "dg2_set_boundary": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32]),
    "dg2_set_inflow_hydrograph": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double),
                                            c_int32]),
    "dg2_set_level_hydrograph": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double),
                                           c_int32]),
    "dg2_set_rainfall": (c_int32, [c_void_p, c_double, c_double, c_double]),
    "dg2_set_gauges": (c_int32, [c_void_p, POINTER(c_double), c_int32, c_int32]),
    "dg2_set_fixed_dt": (c_int32, [c_void_p, c_double]),
    "dg2_step": (c_int32, [c_void_p, c_int32]),
    "dg2_run_to": (c_int32, [c_void_p, c_double]),
    "dg2_sync": (c_int32, [c_void_p]),
    "dg2_read_gauges": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), c_int32,
                                  POINTER(c_int32)]),
    "dg2_diagnostics": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
    "dg2_diagnostics_noalloc": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int64, c_int32, c_double,
                                          c_double, c_double, c_double, c_void_p, c_void_p]),
    "dg2_time_kernels": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double),
                                   POINTER(c_double)]),
    "dg2_set_launch": (c_int32, [c_void_p, c_int32, c_int32]),
    "dg2_set_step_kernel": (c_int32, [c_void_p, c_int32]),
    "dg2_set_stage_check": (c_int32, [c_void_p, c_int32]),
    "dg2_set_partly_wet_flat": (c_int32, [c_void_p, c_int32]),
    "dg2_autotune": (c_int32, [c_void_p, c_double, POINTER(c_int32)]),
    "dg2_set_tune_cache": (c_int32, [c_void_p, ctypes.c_char_p]),
    "dg2_get_launch": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "dg2_batch_set_tune_cache": (c_int32, [c_void_p, ctypes.c_char_p]),
    "dg2_batch_get_launch": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                       POINTER(c_int32)]),
    "dg2_state_layout": (c_int32, [c_void_p, POINTER(c_size_t), POINTER(c_size_t)]),
    "dg2_bind_device_state": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "dg2_batch_create": (c_int32, [POINTER(c_void_p), c_int32, c_void_p, POINTER(c_void_p)]),
    "dg2_batch_destroy": (None, [c_void_p]),
    "dg2_batch_last_error": (ctypes.c_char_p, [c_void_p]),
    "dg2_batch_refresh": (c_int32, [c_void_p]),
    "dg2_batch_set_launch": (c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    "dg2_batch_autotune": (c_int32, [c_void_p, c_double, POINTER(c_int32)]),
    "dg2_batch_step": (c_int32, [c_void_p, c_int32]),
    "dg2_batch_run_to": (c_int32, [c_void_p, c_double]),
    "dg2_batch_sync": (c_int32, [c_void_p]),
    "dg2_batch_time_steps": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "dg2_adj_create": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_void_p)]),
    "dg2_adj_destroy": (None, [c_void_p]),
    "dg2_adj_last_error": (ctypes.c_char_p, [c_void_p]),
    "dg2_adj_forward": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
    "dg2_adj_backward": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
    "dg2_adj_timing": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double)]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``libdg2.so`` (built by ``python -m paper_2010_02003_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libdg2.so is not built: run `python -m paper_2010_02003_amd.build` "
                           "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return sorted(_SIGS)


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(POINTER(c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Sim:
    """One DG2 simulation context on the current GPU (``dg2_ctx``)."""

    def __init__(self, nx: int, ny: int, dx: float, dy: Optional[float] = None, *,
                 precision: str = "fp64", variant: str = "NL", g: float = 9.81,
                 cfl: float = 0.3, tol_dry: float = 1e-5, ll_threshold: float = 10.0,
                 dt_max: float = 1.0, x0: float = 0.0, y0: float = 0.0, stream=None,
                 flux: str = "HLL"):
        self._lib = load_library()
        self._ctx = c_void_p()
        cfg = Config()
        self._lib.dg2_config_default(byref(cfg), nx, ny, dx, dx if dy is None else dy)
        cfg.prec = {"fp64": FP64, "fp32": FP32}[precision]
        cfg.variant = {"NL": NL, "LL": LL}[variant]
        cfg.flux = {"HLL": FLUX_HLL, "ROE": FLUX_ROE}[flux]
        cfg.g, cfg.cfl, cfg.tol_dry, cfg.ll_threshold, cfg.dt_max = g, cfl, tol_dry, ll_threshold, dt_max
        cfg.x0, cfg.y0 = x0, y0
        if stream == "torch":
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        cfg.hip_stream = stream
        self.cfg = cfg
        self.nx, self.ny = nx, ny
        self.precision = precision
        self.variant = variant
        st = self._lib.dg2_create(byref(cfg), byref(self._ctx))
        if st != 0:
            msg = self._lib.dg2_last_error(None)
            raise DG2Error(st, msg.decode() if msg else "")
        self.ng = 0

    # -- plumbing ----------------------------------------------------------
    def _check(self, st: int):
        if st != 0:
            msg = self._lib.dg2_last_error(self._ctx)
            raise DG2Error(st, msg.decode() if msg else "")

    def close(self):
        if self._ctx:
            self._lib.dg2_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- setup ---------------------------------------------------------------
    def set_dem_corners(self, Z):
        Z = _f64(Z)
        assert Z.shape == (self.ny + 1, self.nx + 1)
        self._check(self._lib.dg2_set_dem_corners(self._ctx, _dp(Z)))

    def set_manning(self, n):
        if np.ndim(n) == 0:
            self._check(self._lib.dg2_set_manning(self._ctx, None, float(n)))
        else:
            a = _f64(n)
            assert a.shape == (self.ny, self.nx)
            self._check(self._lib.dg2_set_manning(self._ctx, _dp(a), 0.0))

    def set_initial_corners(self, surface, is_eta: bool = True, qx=None, qy=None):
        s = _f64(surface)
        qx = None if qx is None else _f64(qx)
        qy = None if qy is None else _f64(qy)
        self._check(self._lib.dg2_set_initial_corners(self._ctx, _dp(s), int(is_eta), _dp(qx), _dp(qy)))

    def set_state(self, modes, t: float = 0.0):
        m = _f64(modes)
        assert m.size == 9 * self.nx * self.ny
        self._check(self._lib.dg2_set_state(self._ctx, _dp(m), float(t)))

    def get_state(self):
        m = np.empty((9, self.ny, self.nx), dtype=np.float64)
        t, step, ldt = c_double(), c_int64(), c_double()
        self._check(self._lib.dg2_get_state(self._ctx, _dp(m), byref(t), byref(step), byref(ldt)))
        return m, t.value, step.value, ldt.value

    def time(self):
        t, step, ldt = c_double(), c_int64(), c_double()
        self._check(self._lib.dg2_get_state(self._ctx, None, byref(t), byref(step), byref(ldt)))
        return t.value, step.value, ldt.value

    def set_boundary(self, side: int, bc: int, first: int = 0, last: int = 0):
        self._check(self._lib.dg2_set_boundary(self._ctx, side, bc, first, last))

    def set_inflow_hydrograph(self, side: int, t, Q):
        t = _f64(t)
        Q = _f64(Q)
        self._check(self._lib.dg2_set_inflow_hydrograph(self._ctx, side, _dp(t), _dp(Q), len(t)))

    def set_level_hydrograph(self, side: int, t, eta):
        t = _f64(t)
        eta = _f64(eta)
        self._check(self._lib.dg2_set_level_hydrograph(self._ctx, side, _dp(t), _dp(eta), len(t)))

    def set_rainfall(self, rate: float, t_begin: float, t_end: float):
        self._check(self._lib.dg2_set_rainfall(self._ctx, rate, t_begin, t_end))

    def set_gauges(self, xy, capacity: int = 0):
        xy = _f64(xy).reshape(-1, 2)
        self._check(self._lib.dg2_set_gauges(self._ctx, _dp(xy), len(xy), capacity))
        self.ng = len(xy)

    def set_fixed_dt(self, dt: float):
        self._check(self._lib.dg2_set_fixed_dt(self._ctx, dt))

    def set_launch(self, rows_per_wave: int, waves_per_block: int = 4):
        self._check(self._lib.dg2_set_launch(self._ctx, rows_per_wave, waves_per_block))

    def set_step_kernel(self, fused: bool):
        self._check(self._lib.dg2_set_step_kernel(self._ctx, 1 if fused else 0))

    def set_stage_check(self, repeats: int):
        self._check(self._lib.dg2_set_stage_check(self._ctx, repeats))

    def set_partly_wet_flat(self, on: bool):
        self._check(self._lib.dg2_set_partly_wet_flat(self._ctx, 1 if on else 0))

    def autotune(self, budget_ms: float = 200.0) -> int:
        r = c_int32()
        self._check(self._lib.dg2_autotune(self._ctx, budget_ms, byref(r)))
        return r.value

    def set_tune_cache(self, path: Optional[str]):
        self._check(self._lib.dg2_set_tune_cache(self._ctx, path.encode() if path else None))

    def get_launch(self):
        """(rows per wavefront, wavefronts per workgroup, taken from the tune cache)."""
        r, w, f = c_int32(), c_int32(), c_int32()
        self._check(self._lib.dg2_get_launch(self._ctx, byref(r), byref(w), byref(f)))
        return r.value, w.value, bool(f.value)

    # -- run -------------------------------------------------------------------
    def step(self, nsteps: int = 1):
        self._check(self._lib.dg2_step(self._ctx, nsteps))

    def run_to(self, T: float):
        self._check(self._lib.dg2_run_to(self._ctx, T))

    def sync(self):
        self._check(self._lib.dg2_sync(self._ctx))

    def read_gauges(self, max_samples: int = 1 << 20):
        if self.ng == 0:
            return np.zeros((0, 0, 4)), np.zeros(0)
        chunks, times = [], []
        while True:
            cap = 4096
            out = np.empty((cap, self.ng, 4), dtype=np.float64)
            t = np.empty(cap, dtype=np.float64)
            ns = c_int32()
            self._check(self._lib.dg2_read_gauges(self._ctx, _dp(out), _dp(t), cap, byref(ns)))
            chunks.append(out[:ns.value])
            times.append(t[:ns.value])
            if ns.value < cap or sum(len(c) for c in chunks) >= max_samples:
                break
        return np.concatenate(chunks), np.concatenate(times)

    def diagnostics(self):
        m, e, h = c_double(), c_double(), c_double()
        self._check(self._lib.dg2_diagnostics(self._ctx, byref(m), byref(e), byref(h)))
        return m.value, e.value, h.value

    def history(self, times):
        """Run to each of the increasing times in turn and record the mass,
        total energy (Eq. 11-12) and smallest mean depth there: an array
        (len(times), 4) of t, mass, energy, min_h."""
        out = np.empty((len(times), 4), dtype=np.float64)
        for k, T in enumerate(times):
            self.run_to(float(T))
            out[k, 0] = self.time()[0]
            out[k, 1:] = self.diagnostics()
        return out

    def time_kernels(self, nsteps: int):
        a, b, w = c_double(), c_double(), c_double()
        self._check(self._lib.dg2_time_kernels(self._ctx, nsteps, byref(a), byref(b), byref(w)))
        return a.value, b.value, w.value

    def state_layout(self):
        b, s = c_size_t(), c_size_t()
        self._check(self._lib.dg2_state_layout(self._ctx, byref(b), byref(s)))
        return b.value, s.value

    def bind_device_state(self, ptr: Optional[int], nbytes: int = 0):
        self._check(self._lib.dg2_bind_device_state(self._ctx, ptr, nbytes))


def diagnostics_noalloc(state_ptr: int, bed_ptr: int, nx: int, ny: int, plane_stride: int,
                        precision: str, dx: float, dy: float, g: float, tol_dry: float,
                        out4_ptr: int, stream_ptr: Optional[int] = None):
    """``dg2_diagnostics_noalloc``: queue the mass/energy/min-depth reduction of
    device planes into four device doubles at ``out4_ptr`` (pointers are
    device addresses, e.g. ``tensor.data_ptr()``).  Allocates nothing."""
    lib = load_library()
    st = lib.dg2_diagnostics_noalloc(state_ptr, bed_ptr, nx, ny, plane_stride,
                                     1 if precision == "fp32" else 0, dx, dy, g, tol_dry,
                                     out4_ptr, stream_ptr)
    if st != 0:
        msg = lib.dg2_last_error(None)
        raise DG2Error(st, msg.decode() if msg else "")


class Batch:
    """Batched ensemble of ``Sim`` members advanced together (``dg2_batch``).

    The members stay owned by the caller and must outlive the batch; step them
    only through it, and call ``sync`` before reading a member.
    """

    def __init__(self, members: Sequence[Sim], stream=None):
        self._lib = load_library()
        self._b = c_void_p()
        self.members = list(members)
        if stream == "torch":
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        arr = (c_void_p * len(self.members))(*[m._ctx.value for m in self.members])
        st = self._lib.dg2_batch_create(arr, len(self.members), stream, byref(self._b))
        if st != 0:
            msg = self._lib.dg2_batch_last_error(None)
            raise DG2Error(st, msg.decode() if msg else "")

    def _check(self, st: int):
        if st != 0:
            msg = self._lib.dg2_batch_last_error(self._b)
            raise DG2Error(st, msg.decode() if msg else "")

    def close(self):
        if self._b:
            self._lib.dg2_batch_destroy(self._b)
            self._b = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refresh(self):
        self._check(self._lib.dg2_batch_refresh(self._b))

    def set_launch(self, rows_per_wave: int = 0, waves_per_block: int = 4, graph_steps: int = 16):
        self._check(self._lib.dg2_batch_set_launch(self._b, rows_per_wave, waves_per_block, graph_steps))

    def autotune(self, budget_ms: float = 500.0) -> int:
        r = c_int32()
        self._check(self._lib.dg2_batch_autotune(self._b, budget_ms, byref(r)))
        return r.value

    def set_tune_cache(self, path: Optional[str]):
        self._check(self._lib.dg2_batch_set_tune_cache(self._b, path.encode() if path else None))

    def get_launch(self):
        """(rows per wavefront, wavefronts per workgroup, graph length, taken from the tune cache)."""
        r, w, g, f = c_int32(), c_int32(), c_int32(), c_int32()
        self._check(self._lib.dg2_batch_get_launch(self._b, byref(r), byref(w), byref(g), byref(f)))
        return r.value, w.value, g.value, bool(f.value)

    def step(self, nsteps: int = 1):
        self._check(self._lib.dg2_batch_step(self._b, nsteps))

    def run_to(self, T: float):
        self._check(self._lib.dg2_batch_run_to(self._b, T))

    def sync(self):
        self._check(self._lib.dg2_batch_sync(self._b))

    def time_steps(self, nsteps: int) -> float:
        ms = c_double()
        self._check(self._lib.dg2_batch_time_steps(self._b, nsteps, byref(ms)))
        return ms.value


class Adjoint:
    """Reverse-mode runner of a ``Sim`` (``dg2_adj``): gauge depths after each
    of ``steps`` fixed-size steps from the Sim's current state, and the
    gradients of a loss on them with respect to the per-cell Manning field and
    the samples of the control side's hydrograph.  The Sim must outlive it."""

    def __init__(self, sim: Sim, steps: int, checkpoint_every: int = 100,
                 control_side: int = -1, n_hydrograph: int = 0):
        self._lib = load_library()
        self.sim = sim
        self.steps = steps
        self.ng = sim.ng
        self.n_hydrograph = n_hydrograph
        self._a = c_void_p()
        # forward runs so far: the library keeps the checkpoints of the last one only
        self.generation = 0
        st = self._lib.dg2_adj_create(sim._ctx, steps, checkpoint_every, control_side, byref(self._a))
        if st != 0:
            msg = self._lib.dg2_adj_last_error(None)
            raise DG2Error(st, msg.decode() if msg else "")

    def _check(self, st: int):
        if st != 0:
            msg = self._lib.dg2_adj_last_error(self._a)
            raise DG2Error(st, msg.decode() if msg else "")

    def close(self):
        if self._a:
            self._lib.dg2_adj_destroy(self._a)
            self._a = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, n_cell=None, Q=None) -> np.ndarray:
        n = None if n_cell is None else _f64(n_cell)
        if n is not None:
            assert n.shape == (self.sim.ny, self.sim.nx)
        q = None if Q is None else _f64(Q)
        if q is not None:
            assert q.shape == (self.n_hydrograph,)
        h = np.empty((self.steps, self.ng), dtype=np.float64)
        self._check(self._lib.dg2_adj_forward(self._a, _dp(n), _dp(q), _dp(h)))
        self.generation += 1
        return h

    def backward(self, dL_dh):
        d = _f64(dL_dh)
        assert d.shape == (self.steps, self.ng)
        gn = np.empty((self.sim.ny, self.sim.nx), dtype=np.float64)
        gq = np.empty(max(self.n_hydrograph, 1), dtype=np.float64)
        self._check(self._lib.dg2_adj_backward(self._a, _dp(d), _dp(gn), _dp(gq)))
        return gn, gq[:self.n_hydrograph]

    def timing(self):
        f, b = c_double(), c_double()
        self._check(self._lib.dg2_adj_timing(self._a, byref(f), byref(b)))
        return f.value, b.value


def sim_from_scenario(sc, stream=None, precision: Optional[str] = None,
                      variant: Optional[str] = None) -> Sim:
    """A ``Sim`` loaded with a ``workloads.Scenario`` (argument marshalling only)."""
    s = Sim(sc.nx, sc.ny, sc.dx, sc.dy, precision=precision or sc.precision,
            variant=variant or sc.variant, g=sc.g, cfl=sc.cfl, tol_dry=sc.tol_dry,
            ll_threshold=sc.theta, dt_max=sc.dt_max, x0=sc.x0, y0=sc.y0, stream=stream,
            flux=sc.flux)
    s.set_dem_corners(sc.Z)
    s.set_manning(sc.manning)
    for b in sc.inflows:
        s.set_boundary(b.side, BC_INFLOW_Q, b.first, b.last)
        s.set_inflow_hydrograph(b.side, b.t, b.Q)
    for b in sc.levels:
        s.set_boundary(b.side, BC_LEVEL, b.first, b.last)
        s.set_level_hydrograph(b.side, b.t, b.eta)
    for side, first, last in sc.opens:
        s.set_boundary(side, BC_OPEN, first, last)
    if sc.rain is not None:
        s.set_rainfall(*sc.rain)
    if sc.fixed_dt > 0:
        s.set_fixed_dt(sc.fixed_dt)
    if sc.stage_check > 0:
        s.set_stage_check(sc.stage_check)
    if sc.partly_wet_flat:
        s.set_partly_wet_flat(True)
    s.set_initial_corners(sc.surface, sc.is_eta, sc.qx, sc.qy)
    if sc.gauges is not None:
        s.set_gauges(sc.gauges)
    return s
