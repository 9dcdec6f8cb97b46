"""ctypes binding of ``liblbm.so`` (declared in include/lbm.h).

Argument marshalling only: every step of the lattice update, the monitors and
the transfers run in the library's HIP kernels.  Functions keep the C names
(``lbm_create``, ``lbm_step``, ...) and raise :class:`LbmError` on a non-zero
return; :class:`Cavity` wraps a handle.  Host arrays are NumPy float64;
device arrays and streams may be torch objects (``data_ptr()`` /
``cuda_stream``), torch itself is not needed otherwise.

The library must have been built (``python paper_2211_05009_amd/build.py``);
importing this module without it raises ImportError: there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_EIO, LBM_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
LBM_F64, LBM_F32_SHIFTED = 0, 1
LBM_OPT_USE_GRAPH, LBM_OPT_STEP_VARIANT, LBM_OPT_NUM_VARIANTS, LBM_OPT_GRAPH_STEPS = 1, 2, 3, 4
LBM_OPT_STEPS_PER_LAUNCH, LBM_OPT_TILE_X, LBM_OPT_TILE_Y, LBM_OPT_SYNC = 5, 6, 7, 8
LBM_INIT_RENORMALISE_MASS, LBM_INIT_ZERO_STAGGERED = 1, 2
LBM_WALL_BOUNCE_BACK, LBM_WALL_NEE = 0, 1
WALLS = {"bounce-back": LBM_WALL_BOUNCE_BACK, "nee": LBM_WALL_NEE}
DTYPES = {"f64": LBM_F64, "f32s": LBM_F32_SHIFTED}

_ERRNAMES = {LBM_EINVAL: "LBM_EINVAL", LBM_ENOMEM: "LBM_ENOMEM",
             LBM_EDEVICE: "LBM_EDEVICE", LBM_EUNSTABLE: "LBM_EUNSTABLE",
             LBM_EIO: "LBM_EIO", LBM_ESTATE: "LBM_ESTATE"}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class lbm_info_t(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("pitch", ct.c_int),
                ("dtype", ct.c_int), ("re", ct.c_double), ("u_lid", ct.c_double),
                ("tau", ct.c_double), ("omega", ct.c_double),
                ("steps_done", ct.c_int64), ("device_bytes", ct.c_size_t),
                ("wall", ct.c_int)]


class lbm_launch_record_t(ct.Structure):
    _fields_ = [("steps", ct.c_int64), ("multi_variant", ct.c_int),
                ("steps_per_launch", ct.c_int), ("multi_launches", ct.c_int64),
                ("multi_monitor_launches", ct.c_int64), ("single_variant", ct.c_int),
                ("single_launches", ct.c_int64), ("graph_replays", ct.c_int64),
                ("monitor_passes", ct.c_int64), ("probe_launches", ct.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _load():
    # PyTorch ROCm wheels bundle their own HIP runtime under the same soname
    # as ROCm's (libamdhip64.so.7).  Loading torch first makes that one
    # runtime serve both torch and this library, so torch streams and device
    # pointers handed to the library belong to the runtime that launches its
    # kernels.  Without torch, ROCm's runtime is used.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2211_05009_amd/build.py` (no CPU fallback)")
    return ct.CDLL(LIB_PATH)


_lib = _load()
_h = ct.c_void_p
_dp = ct.POINTER(ct.c_double)
_i64 = ct.c_int64

# name -> argtypes (all return int unless listed in _RESTYPES)
SIGNATURES = {
    "lbm_last_error": [],
    "lbm_version": [],
    "lbm_create": [ct.c_int, ct.c_int, ct.c_double, ct.c_double, ct.c_int, ct.POINTER(_h)],
    "lbm_create_tau": [ct.c_int, ct.c_int, ct.c_double, ct.c_double, ct.c_int, ct.POINTER(_h)],
    "lbm_create_wall": [ct.c_int, ct.c_int, ct.c_double, ct.c_double, ct.c_int, ct.c_int,
                        ct.POINTER(_h)],
    "lbm_destroy": [_h],
    "lbm_set_stream": [_h, ct.c_void_p],
    "lbm_info": [_h, ct.POINTER(lbm_info_t)],
    "lbm_set_option": [_h, ct.c_int, _i64],
    "lbm_get_option": [_h, ct.c_int, ct.POINTER(_i64)],
    "lbm_step": [_h, _i64],
    "lbm_last_launches": [_h, ct.POINTER(lbm_launch_record_t)],
    "lbm_steps_done": [_h, ct.POINTER(_i64)],
    "lbm_moments": [_h, ct.c_void_p, ct.c_void_p, ct.c_void_p],
    "lbm_moments_device": [_h, ct.c_void_p, ct.c_void_p, ct.c_void_p],
    "lbm_probe": [_h, ct.c_int, ct.c_void_p, ct.c_void_p],
    "lbm_probe_config": [_h, ct.c_int, ct.c_void_p, ct.c_int, _i64],
    "lbm_probe_read": [_h, ct.c_void_p, _i64, ct.POINTER(_i64)],
    "lbm_mass": [_h, _dp],
    "lbm_residual": [_h, _dp, ct.POINTER(_i64)],
    "lbm_stream_function": [_h, ct.c_void_p],
    "lbm_classify_series": [ct.c_void_p, ct.c_int, _i64, _i64, ct.c_double, ct.c_double,
                            ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p],
    "lbm_classify_series_noalloc": [ct.c_void_p, ct.c_int, _i64, _i64, ct.c_double,
                                    ct.c_double, ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p],
    "lbm_probe_classify": [_h, ct.c_int, _i64, ct.c_double, ct.c_double, ct.c_int, ct.c_int,
                           ct.c_void_p],
    "lbm_vortex_extrema": [_h, ct.c_void_p],
    "lbm3d_create": [ct.c_int, ct.c_int, ct.c_int, ct.c_double, ct.c_double, ct.c_int,
                     ct.POINTER(_h)],
    "lbm3d_destroy": [_h],
    "lbm3d_set_stream": [_h, ct.c_void_p],
    "lbm3d_set_option": [_h, ct.c_int, _i64],
    "lbm3d_get_option": [_h, ct.c_int, ct.POINTER(_i64)],
    "lbm3d_step": [_h, _i64],
    "lbm3d_steps_done": [_h, ct.POINTER(_i64)],
    "lbm3d_residual": [_h, ct.POINTER(ct.c_double), ct.POINTER(_i64)],
    "lbm3d_mass": [_h, ct.POINTER(ct.c_double)],
    "lbm3d_moments": [_h, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p],
    "lbm3d_set_populations": [_h, ct.c_void_p],
    "lbm3d_get_populations": [_h, ct.c_void_p],
    "lbm3d_autotune": [_h, ct.c_int, ct.POINTER(ct.c_int), ct.POINTER(ct.c_double)],
    "lbm_vortex_centres": [_h, ct.c_double, ct.c_int, ct.c_void_p, ct.POINTER(ct.c_int)],
    "lbm_bottom_vortex_count": [_h, ct.c_double, ct.POINTER(ct.c_int)],
    "lbm_set_populations": [_h, ct.c_void_p],
    "lbm_get_populations": [_h, ct.c_void_p],
    "lbm_init_fields": [_h, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int],
    "lbm_save": [_h, ct.c_char_p],
    "lbm_load": [_h, ct.c_char_p],
    "lbm_autotune": [_h, ct.c_int, ct.c_int, ct.POINTER(ct.c_int), _dp],
    "lbm_batch_create": [ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_double,
                         ct.c_int, ct.POINTER(_h)],
    "lbm_batch_destroy": [_h],
    "lbm_batch_set_stream": [_h, ct.c_void_p],
    "lbm_batch_set_option": [_h, ct.c_int, _i64],
    "lbm_batch_get_option": [_h, ct.c_int, ct.POINTER(_i64)],
    "lbm_batch_step": [_h, _i64],
    "lbm_batch_set_threshold": [_h, ct.c_double],
    "lbm_batch_set_active": [_h, ct.c_int, ct.c_int],
    "lbm_batch_status": [_h, ct.c_int, ct.POINTER(_i64), _dp, ct.POINTER(_i64),
                         ct.POINTER(ct.c_int)],
    "lbm_batch_mass": [_h, ct.c_int, _dp],
    "lbm_batch_moments": [_h, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p],
    "lbm_batch_get_populations": [_h, ct.c_int, ct.c_void_p],
    "lbm_batch_set_populations": [_h, ct.c_int, ct.c_void_p],
    "lbm_batch_init_fields": [_h, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int],
    "lbm_batch_info": [_h, ct.POINTER(ct.c_int), ct.POINTER(_i64), ct.POINTER(_i64),
                       ct.POINTER(ct.c_size_t)],
    "lbm_batch_autotune": [_h, ct.c_int, ct.c_int, ct.POINTER(ct.c_int), _dp],
    "lbm_init_fields_device": [_h, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int],
    "lbm_batch_init_fields_device": [_h, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                     ct.c_int],
    "lbm_batch_cavity": [_h, ct.c_int, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), _dp, _dp],
    "lbm_batch_residuals": [_h, ct.c_void_p],
    "lbm_batch_probe_config": [_h, ct.c_int, ct.c_void_p, _i64],
    "lbm_batch_probe_read": [_h, ct.c_int, ct.c_void_p, _i64, ct.POINTER(_i64),
                             ct.POINTER(_i64)],
    "lbm_batch_probe_classify": [_h, ct.c_int, _i64, ct.c_double, ct.c_double, ct.c_int,
                                 ct.c_int, ct.c_void_p],
    "lbm_batch_canvas": [_h, ct.c_int, ct.c_void_p, ct.c_void_p],
    "lbm_sur_create": [ct.c_int, ct.POINTER(_h)],
    "lbm_sur_destroy": [_h],
    "lbm_sur_set_stream": [_h, ct.c_void_p],
    "lbm_sur_num_params": [_h, ct.POINTER(_i64)],
    "lbm_sur_set_params": [_h, ct.c_void_p, _i64],
    "lbm_sur_get_params": [_h, ct.c_void_p, ct.c_void_p],
    "lbm_sur_init_params": [_h, ct.c_void_p, _i64],
    "lbm_sur_forward": [_h, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p],
    "lbm_sur_train_step": [_h, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                           ct.c_double, ct.c_int, _dp],
    "lbm_sur_warm_start": [_h, _h],
    "lbm_sur_warm_start_batch": [_h, _h, ct.c_int],
    "lbm_nn_conv3x3": [ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                       ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p, ct.c_int, ct.c_int,
                       ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_int,
                       ct.c_int, ct.c_void_p],
    "lbm_nn_bias_grad": [ct.c_int, ct.c_int, ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p,
                         ct.c_void_p],
    "lbm_nn_pool2": [ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_void_p, ct.c_int,
                     ct.c_int, ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_void_p],
    "lbm_nn_up2": [ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_void_p, ct.c_int,
                   ct.c_int, ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p],
}
_RESTYPES = {"lbm_last_error": ct.c_char_p, "lbm_version": ct.c_char_p}

for _name, _args in SIGNATURES.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _RESTYPES.get(_name, ct.c_int)


def _check(rc):
    if rc != LBM_OK:
        raise LbmError(rc, _lib.lbm_last_error().decode())
    return rc


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


# ---------------------------------------------------------------- C names ---
def lbm_last_error():
    return _lib.lbm_last_error().decode()


def lbm_version():
    return _lib.lbm_version().decode()


def lbm_create(nx, ny, re, u_lid, dtype):
    h = _h()
    _check(_lib.lbm_create(int(nx), int(ny), float(re), float(u_lid),
                           DTYPES.get(dtype, dtype), ct.byref(h)))
    return h


def lbm_create_tau(nx, ny, tau, u_lid, dtype):
    h = _h()
    _check(_lib.lbm_create_tau(int(nx), int(ny), float(tau), float(u_lid),
                               DTYPES.get(dtype, dtype), ct.byref(h)))
    return h


def lbm_create_wall(nx, ny, re, u_lid, dtype, wall):
    h = _h()
    _check(_lib.lbm_create_wall(int(nx), int(ny), float(re), float(u_lid),
                                DTYPES.get(dtype, dtype), WALLS.get(wall, wall), ct.byref(h)))
    return h


def lbm_destroy(h):
    _check(_lib.lbm_destroy(h))


def _stream_ptr(stream):
    """A torch.cuda.Stream, a raw hipStream_t integer, or None -> c_void_p."""
    raw = getattr(stream, "cuda_stream", stream)
    return ct.c_void_p(raw) if raw else None


def lbm_set_stream(h, stream):
    """``stream``: a torch.cuda.Stream, a raw hipStream_t integer, or None."""
    _check(_lib.lbm_set_stream(h, _stream_ptr(stream)))


def lbm_info(h):
    info = lbm_info_t()
    _check(_lib.lbm_info(h, ct.byref(info)))
    return {k: getattr(info, k) for k, _ in lbm_info_t._fields_}


def lbm_set_option(h, option, value):
    _check(_lib.lbm_set_option(h, int(option), int(value)))


def lbm_get_option(h, option):
    v = _i64()
    _check(_lib.lbm_get_option(h, int(option), ct.byref(v)))
    return v.value


def lbm_step(h, n):
    _check(_lib.lbm_step(h, int(n)))


def lbm_last_launches(h):
    """What the last lbm_step call launched (a dict of the record's fields)."""
    rec = lbm_launch_record_t()
    _check(_lib.lbm_last_launches(h, ct.byref(rec)))
    return rec.as_dict()


def lbm_steps_done(h):
    t = _i64()
    _check(_lib.lbm_steps_done(h, ct.byref(t)))
    return t.value


def lbm_moments(h, nx, ny):
    rho, ux, uy = (np.empty((ny, nx)) for _ in range(3))
    _check(_lib.lbm_moments(h, _ptr(rho), _ptr(ux), _ptr(uy)))
    return rho, ux, uy


def lbm_moments_device(h, rho, ux, uy):
    """Device outputs: torch float64 tensors (or raw pointers / None)."""
    ptrs = [None if a is None else ct.c_void_p(a.data_ptr() if hasattr(a, "data_ptr") else a)
            for a in (rho, ux, uy)]
    _check(_lib.lbm_moments_device(h, *ptrs))


def lbm_probe(h, points):
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    out = np.empty((pts.shape[0], 3))
    _check(_lib.lbm_probe(h, pts.shape[0], _ptr(pts), _ptr(out)))
    return out


def lbm_probe_config(h, points, every, capacity):
    if points is None or len(points) == 0:
        _check(_lib.lbm_probe_config(h, 0, None, int(every), int(capacity)))
        return
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    _check(_lib.lbm_probe_config(h, pts.shape[0], _ptr(pts), int(every), int(capacity)))


def lbm_probe_read(h, npts, max_records):
    buf = np.empty((max(int(max_records), 1), 1 + 3 * npts))
    n = _i64()
    _check(_lib.lbm_probe_read(h, _ptr(buf), int(max_records), ct.byref(n)))
    return buf[:n.value]


def lbm_mass(h):
    m = ct.c_double()
    _check(_lib.lbm_mass(h, ct.byref(m)))
    return m.value


def lbm_residual(h):
    r = ct.c_double()
    t = _i64()
    _check(_lib.lbm_residual(h, ct.byref(r), ct.byref(t)))
    return r.value, t.value


def lbm_stream_function(h, nx, ny):
    psi = np.empty((ny, nx))
    _check(_lib.lbm_stream_function(h, _ptr(psi)))
    return psi


LBM_FLOW_TOO_SHORT, LBM_FLOW_STEADY, LBM_FLOW_PERIODIC, LBM_FLOW_APERIODIC, LBM_FLOW_DRIFT = \
    -1, 0, 1, 2, 3
FLOW_STATES = {LBM_FLOW_TOO_SHORT: "too short", LBM_FLOW_STEADY: "steady",
               LBM_FLOW_PERIODIC: "periodic", LBM_FLOW_APERIODIC: "aperiodic",
               LBM_FLOW_DRIFT: "drift"}


class FlowState(ct.Structure):
    """lbm_flow_state_t."""
    _fields_ = [("state", ct.c_int), ("lag", ct.c_int), ("period", ct.c_double),
                ("amplitude", ct.c_double), ("mean", ct.c_double), ("std", ct.c_double),
                ("mismatch", ct.c_double), ("cycle", ct.c_double),
                ("cycle_mismatch", ct.c_double)]

    def as_dict(self):
        return {"state": FLOW_STATES[self.state], "lag": self.lag, "period": self.period,
                "amplitude": self.amplitude, "mean": self.mean, "std": self.std,
                "mismatch": self.mismatch, "cycle": self.cycle,
                "cycle_mismatch": self.cycle_mismatch}


def lbm_classify_series(series_dev, steady_tol, periodic_tol, min_lag=1, max_lag=0,
                        stream=None):
    """series_dev: a 2-D FP64 device tensor [nseries, n] (rows contiguous)."""
    ns, n = int(series_dev.shape[0]), int(series_dev.shape[1])
    if series_dev.stride(1) != 1:
        raise ValueError("rows must be contiguous")
    out = (FlowState * ns)()
    _check(_lib.lbm_classify_series(ct.c_void_p(series_dev.data_ptr()), ns, n,
                                    int(series_dev.stride(0)), float(steady_tol),
                                    float(periodic_tol), int(min_lag), int(max_lag), out,
                                    _stream_ptr(stream)))
    return [o.as_dict() for o in out]


def lbm_classify_series_noalloc(series_dev, steady_tol, periodic_tol, out_dev, min_lag=1,
                                max_lag=0, stream=None):
    """lbm_classify_series into out_dev, a device tensor of at least
    nseries * sizeof(FlowState) bytes, issued on `stream` without allocating
    or synchronising (read out_dev after the stream has finished; see
    flow_states_from_bytes)."""
    ns, n = int(series_dev.shape[0]), int(series_dev.shape[1])
    if series_dev.stride(1) != 1:
        raise ValueError("rows must be contiguous")
    if out_dev.numel() * out_dev.element_size() < ns * ct.sizeof(FlowState):
        raise ValueError(f"out_dev holds fewer than {ns} records")
    _check(_lib.lbm_classify_series_noalloc(
        ct.c_void_p(series_dev.data_ptr()), ns, n, int(series_dev.stride(0)),
        float(steady_tol), float(periodic_tol), int(min_lag), int(max_lag),
        ct.c_void_p(out_dev.data_ptr()), _stream_ptr(stream)))


def flow_states_from_bytes(raw, n):
    """The first n lbm_flow_state_t records of a host byte buffer, as dicts."""
    recs = (FlowState * n).from_buffer_copy(bytes(raw[:n * ct.sizeof(FlowState)]))
    return [r.as_dict() for r in recs]


def lbm_probe_classify(h, npts, component, window, steady_tol, periodic_tol, min_lag=1,
                       max_lag=0):
    out = (FlowState * int(npts))()
    _check(_lib.lbm_probe_classify(h, int(component), int(window), float(steady_tol),
                                   float(periodic_tol), int(min_lag), int(max_lag), out))
    return [o.as_dict() for o in out]


class Vortex(ct.Structure):
    """lbm_vortex_t: Psi (lattice units), centre (x, y) in units of the
    width, site indices and kind (+1 maximum of Psi, -1 minimum)."""
    _fields_ = [("psi", ct.c_double), ("x", ct.c_double), ("y", ct.c_double),
                ("ix", ct.c_int), ("iy", ct.c_int), ("kind", ct.c_int), ("reserved", ct.c_int)]

    def as_tuple(self):
        return (self.iy, self.ix, self.kind, self.psi)


def lbm_vortex_extrema(h):
    """[primary, lower_left, lower_right] as Vortex records."""
    out = (Vortex * 3)()
    _check(_lib.lbm_vortex_extrema(h, out))
    return list(out)


def lbm_vortex_centres(h, min_abs_psi=0.0, cap=4096):
    """(list of the first min(count, cap) Vortex records in row-major order,
    total count)."""
    out = (Vortex * max(int(cap), 1))()
    n = ct.c_int()
    _check(_lib.lbm_vortex_centres(h, float(min_abs_psi), int(cap), out if cap > 0 else None,
                                   ct.byref(n)))
    return list(out[:min(n.value, int(cap))]), n.value


def lbm_bottom_vortex_count(h, min_abs_psi=0.0):
    n = ct.c_int()
    _check(_lib.lbm_bottom_vortex_count(h, float(min_abs_psi), ct.byref(n)))
    return n.value


def lbm_set_populations(h, f, nx, ny):
    f = _f64(f, (9, ny, nx))
    _check(_lib.lbm_set_populations(h, _ptr(f)))


def lbm_get_populations(h, nx, ny):
    f = np.empty((9, ny, nx))
    _check(_lib.lbm_get_populations(h, _ptr(f)))
    return f


def _init_flags(renormalise_mass, zero_staggered):
    return (LBM_INIT_RENORMALISE_MASS if renormalise_mass else 0) | \
        (LBM_INIT_ZERO_STAGGERED if zero_staggered else 0)


def lbm_init_fields(h, rho, ux, uy, nx, ny, renormalise_mass=True, zero_staggered=False):
    arrs = [None if a is None else _f64(a, (ny, nx)) for a in (rho, ux, uy)]
    _check(_lib.lbm_init_fields(h, *[_ptr(a) for a in arrs],
                                _init_flags(renormalise_mass, zero_staggered)))


def lbm_save(h, path):
    _check(_lib.lbm_save(h, os.fsencode(path)))


def lbm_load(h, path):
    _check(_lib.lbm_load(h, os.fsencode(path)))


def lbm_autotune(h, chunks, use_cache=True):
    best = ct.c_int()
    ms = ct.c_double()
    _check(_lib.lbm_autotune(h, int(chunks), int(bool(use_cache)), ct.byref(best), ct.byref(ms)))
    return best.value, ms.value


# ----------------------------------------------------------------- batch ---
def lbm_batch_create(nx, ny, re, u_lid, dtype):
    nx = np.ascontiguousarray(nx, dtype=np.int32)
    ny = np.ascontiguousarray(ny, dtype=np.int32)
    re = np.ascontiguousarray(re, dtype=np.float64)
    if not (nx.shape == ny.shape == re.shape and nx.ndim == 1):
        raise ValueError("nx, ny, re must be 1-D arrays of one length")
    b = _h()
    _check(_lib.lbm_batch_create(len(nx), _ptr(nx), _ptr(ny), _ptr(re), float(u_lid),
                                 DTYPES.get(dtype, dtype), ct.byref(b)))
    return b


def lbm_batch_destroy(b):
    _check(_lib.lbm_batch_destroy(b))


def lbm_batch_set_stream(b, stream):
    raw = getattr(stream, "cuda_stream", stream)
    _check(_lib.lbm_batch_set_stream(b, ct.c_void_p(raw) if raw else None))


def lbm_batch_set_option(b, option, value):
    _check(_lib.lbm_batch_set_option(b, int(option), int(value)))


def lbm_batch_get_option(b, option):
    v = _i64()
    _check(_lib.lbm_batch_get_option(b, int(option), ct.byref(v)))
    return v.value


def lbm_batch_step(b, n):
    _check(_lib.lbm_batch_step(b, int(n)))


def lbm_batch_set_threshold(b, residual):
    _check(_lib.lbm_batch_set_threshold(b, float(residual)))


def lbm_batch_set_active(b, k, active):
    _check(_lib.lbm_batch_set_active(b, int(k), int(bool(active))))


def lbm_batch_status(b, k):
    t, r, rt, a = _i64(), ct.c_double(), _i64(), ct.c_int()
    _check(_lib.lbm_batch_status(b, int(k), ct.byref(t), ct.byref(r), ct.byref(rt), ct.byref(a)))
    return {"steps_done": t.value, "residual": r.value, "residual_step": rt.value,
            "active": bool(a.value)}


def lbm_batch_mass(b, k):
    m = ct.c_double()
    _check(_lib.lbm_batch_mass(b, int(k), ct.byref(m)))
    return m.value


def lbm_batch_moments(b, k, nx, ny):
    rho, ux, uy = (np.empty((ny, nx)) for _ in range(3))
    _check(_lib.lbm_batch_moments(b, int(k), _ptr(rho), _ptr(ux), _ptr(uy)))
    return rho, ux, uy


def lbm_batch_get_populations(b, k, nx, ny):
    f = np.empty((9, ny, nx))
    _check(_lib.lbm_batch_get_populations(b, int(k), _ptr(f)))
    return f


def lbm_batch_set_populations(b, k, f, nx, ny):
    f = _f64(f, (9, ny, nx))
    _check(_lib.lbm_batch_set_populations(b, int(k), _ptr(f)))


def lbm_batch_init_fields(b, k, rho, ux, uy, nx, ny, renormalise_mass=True,
                          zero_staggered=False):
    arrs = [None if a is None else _f64(a, (ny, nx)) for a in (rho, ux, uy)]
    _check(_lib.lbm_batch_init_fields(b, int(k), *[_ptr(a) for a in arrs],
                                      _init_flags(renormalise_mass, zero_staggered)))


def lbm_batch_info(b):
    n, sites, t, nbytes = ct.c_int(), _i64(), _i64(), ct.c_size_t()
    _check(_lib.lbm_batch_info(b, ct.byref(n), ct.byref(sites), ct.byref(t), ct.byref(nbytes)))
    return {"n": n.value, "total_sites": sites.value, "steps_done": t.value,
            "device_bytes": nbytes.value}


def lbm_batch_autotune(b, chunks, use_cache=True):
    best = ct.c_int()
    ms = ct.c_double()
    _check(_lib.lbm_batch_autotune(b, int(chunks), int(bool(use_cache)), ct.byref(best),
                                   ct.byref(ms)))
    return best.value, ms.value


def _dptr(t):
    """Device pointer of a torch tensor (or an int / None)."""
    if t is None:
        return None
    return ct.c_void_p(t.data_ptr() if hasattr(t, "data_ptr") else int(t))


def _sptr(stream):
    raw = getattr(stream, "cuda_stream", stream)
    return ct.c_void_p(raw) if raw else None


def lbm_init_fields_device(h, rho, ux, uy, renormalise_mass=True, zero_staggered=False):
    _check(_lib.lbm_init_fields_device(h, _dptr(rho), _dptr(ux), _dptr(uy),
                                       _init_flags(renormalise_mass, zero_staggered)))


def lbm_batch_init_fields_device(b, k, rho, ux, uy, renormalise_mass=True,
                                 zero_staggered=False):
    _check(_lib.lbm_batch_init_fields_device(b, int(k), _dptr(rho), _dptr(ux), _dptr(uy),
                                             _init_flags(renormalise_mass, zero_staggered)))


def lbm_batch_residuals(b, n):
    r = np.empty(int(n))
    _check(_lib.lbm_batch_residuals(b, _ptr(r)))
    return r


def lbm_batch_probe_config(b, xy, capacity):
    """xy: [n, npts, 2] points in units of L (npts = 0 removes the probes)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    npts = int(xy.shape[1]) if xy.ndim == 3 else 0
    _check(_lib.lbm_batch_probe_config(b, npts, _ptr(xy) if npts else None, int(capacity)))
    return npts


def lbm_batch_probe_read(b, k, npts, max_records):
    """(records [m, npts, 3], step of the first record)."""
    buf = np.empty((max(int(max_records), 1), npts, 3))
    n = _i64()
    first = _i64()
    _check(_lib.lbm_batch_probe_read(b, int(k), _ptr(buf), int(max_records), ct.byref(n),
                                     ct.byref(first)))
    return buf[:n.value], first.value


def lbm_batch_probe_classify(b, n, npts, component, window, steady_tol, periodic_tol,
                             min_lag=1, max_lag=0):
    """[n][npts] dicts (state "too short" for cavities with too few records)."""
    out = (FlowState * (int(n) * int(npts)))()
    _check(_lib.lbm_batch_probe_classify(b, int(component), int(window), float(steady_tol),
                                         float(periodic_tol), int(min_lag), int(max_lag), out))
    res = [o.as_dict() for o in out]
    return [res[c * npts:(c + 1) * npts] for c in range(int(n))]


def lbm_batch_cavity(b, k):
    nx, ny, re, u = ct.c_int(), ct.c_int(), ct.c_double(), ct.c_double()
    _check(_lib.lbm_batch_cavity(b, int(k), ct.byref(nx), ct.byref(ny), ct.byref(re),
                                 ct.byref(u)))
    return nx.value, ny.value, re.value, u.value


def lbm_batch_canvas(b, k, target, mask):
    """target: torch FP32 [256, 128, 3] (device), mask: FP32 [256, 128]."""
    _check(_lib.lbm_batch_canvas(b, int(k), _dptr(target), _dptr(mask)))


# -------------------------------------------------------------- surrogate ---
def lbm_sur_create(max_batch):
    s = _h()
    _check(_lib.lbm_sur_create(int(max_batch), ct.byref(s)))
    return s


def lbm_sur_destroy(s):
    _check(_lib.lbm_sur_destroy(s))


def lbm_sur_set_stream(s, stream):
    _check(_lib.lbm_sur_set_stream(s, _sptr(stream)))


def lbm_sur_num_params(s):
    n = _i64()
    _check(_lib.lbm_sur_num_params(s, ct.byref(n)))
    return n.value


def lbm_sur_set_params(s, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(_lib.lbm_sur_set_params(s, _ptr(p), p.size))


def lbm_sur_init_params(s, normals):
    z = np.ascontiguousarray(normals, dtype=np.float32)
    _check(_lib.lbm_sur_init_params(s, _ptr(z), z.size))


def lbm_sur_get_params(s, with_grads=False):
    n = lbm_sur_num_params(s)
    p = np.empty(n, dtype=np.float32)
    g = np.empty(n, dtype=np.float32) if with_grads else None
    _check(_lib.lbm_sur_get_params(s, _ptr(p), _ptr(g)))
    return (p, g) if with_grads else p


def lbm_sur_forward(s, re, ar, out):
    re = np.ascontiguousarray(re, dtype=np.float64)
    ar = np.ascontiguousarray(ar, dtype=np.float64)
    _check(_lib.lbm_sur_forward(s, len(re), _ptr(re), _ptr(ar), _dptr(out)))


def lbm_sur_train_step(s, re, ar, target, mask, lr, apply_update=True):
    re = np.ascontiguousarray(re, dtype=np.float64)
    ar = np.ascontiguousarray(ar, dtype=np.float64)
    loss = ct.c_double()
    _check(_lib.lbm_sur_train_step(s, len(re), _ptr(re), _ptr(ar), _dptr(target), _dptr(mask),
                                   float(lr), int(bool(apply_update)), ct.byref(loss)))
    return loss.value


def lbm_sur_warm_start(s, h):
    _check(_lib.lbm_sur_warm_start(s, h))


def lbm_sur_warm_start_batch(s, b, k):
    _check(_lib.lbm_sur_warm_start_batch(s, b, int(k)))


def lbm_nn_conv3x3(mode, n, h, w, ci, co, x, xs, xo, g, gs, go, wt, bias, relu, out, os_, oo,
                   accumulate=False, stream=None):
    _check(_lib.lbm_nn_conv3x3(int(mode), n, h, w, ci, co, _dptr(x), xs, xo, _dptr(g), gs, go,
                               _dptr(wt), _dptr(bias), int(relu), _dptr(out), os_, oo,
                               int(bool(accumulate)), _sptr(stream)))


def lbm_nn_bias_grad(npix, co, g, gs, go, gb, stream=None):
    _check(_lib.lbm_nn_bias_grad(npix, co, _dptr(g), gs, go, _dptr(gb), _sptr(stream)))


def lbm_nn_pool2(backward, n, h, w, c, x, xs, xo, out, os_, oo, accumulate=False, stream=None):
    _check(_lib.lbm_nn_pool2(int(bool(backward)), n, h, w, c, _dptr(x), xs, xo, _dptr(out), os_,
                             oo, int(bool(accumulate)), _sptr(stream)))


def lbm_nn_up2(backward, n, h, w, c, x, xs, xo, out, os_, oo, stream=None):
    _check(_lib.lbm_nn_up2(int(bool(backward)), n, h, w, c, _dptr(x), xs, xo, _dptr(out), os_,
                           oo, _sptr(stream)))


# ------------------------------------------------------------ convenience ---
class Cavity:
    """A lid-driven cavity on the GPU (one library handle).

    wall: "bounce-back" (half-way walls, nx x ny sites, L = nx) or "nee"
    (non-equilibrium extrapolation on on-node walls, nx x ny nodes,
    L = nx - 1)."""

    def __init__(self, nx, ny, re=None, u_lid=0.1, dtype="f64", tau=None, wall="bounce-back"):
        self.nx, self.ny = int(nx), int(ny)
        self.wall = wall
        if tau is not None:
            if WALLS.get(wall, wall) != LBM_WALL_BOUNCE_BACK:
                raise ValueError("tau= is for half-way walls; give re for wall='nee'")
            self.h = lbm_create_tau(nx, ny, tau, u_lid, dtype)
        elif WALLS.get(wall, wall) != LBM_WALL_BOUNCE_BACK:
            self.h = lbm_create_wall(nx, ny, re, u_lid, dtype, wall)
        else:
            self.h = lbm_create(nx, ny, re, u_lid, dtype)
        self.npts = 0

    def close(self):
        if self.h:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def info(self):
        return lbm_info(self.h)

    @property
    def steps_done(self):
        return lbm_steps_done(self.h)

    def step(self, n=1):
        lbm_step(self.h, n)
        return self

    def last_launches(self):
        return lbm_last_launches(self.h)

    def moments(self):
        return lbm_moments(self.h, self.nx, self.ny)

    def moments_device(self, rho, ux, uy):
        lbm_moments_device(self.h, rho, ux, uy)

    def probe(self, points):
        return lbm_probe(self.h, points)

    def probe_config(self, points, every, capacity):
        lbm_probe_config(self.h, points, every, capacity)
        self.npts = 0 if points is None else len(points)

    def probe_read(self, max_records):
        return lbm_probe_read(self.h, self.npts, max_records)

    def mass(self):
        return lbm_mass(self.h)

    def residual(self):
        return lbm_residual(self.h)

    def stream_function(self):
        return lbm_stream_function(self.h, self.nx, self.ny)

    def probe_classify(self, component, window, steady_tol, periodic_tol, min_lag=1,
                       max_lag=0):
        return lbm_probe_classify(self.h, self.npts, component, window, steady_tol,
                                  periodic_tol, min_lag, max_lag)

    def vortex_extrema(self):
        return lbm_vortex_extrema(self.h)

    def vortex_centres(self, min_abs_psi=0.0, cap=4096):
        return lbm_vortex_centres(self.h, min_abs_psi, cap)

    def bottom_vortex_count(self, min_abs_psi=0.0):
        return lbm_bottom_vortex_count(self.h, min_abs_psi)

    def set_populations(self, f):
        lbm_set_populations(self.h, f, self.nx, self.ny)

    def get_populations(self):
        return lbm_get_populations(self.h, self.nx, self.ny)

    def init_fields(self, rho=None, ux=None, uy=None, renormalise_mass=True,
                    zero_staggered=False):
        lbm_init_fields(self.h, rho, ux, uy, self.nx, self.ny, renormalise_mass,
                        zero_staggered)

    def set_stream(self, stream):
        lbm_set_stream(self.h, stream)

    def set_option(self, option, value):
        lbm_set_option(self.h, option, value)

    def get_option(self, option):
        return lbm_get_option(self.h, option)

    def save(self, path):
        lbm_save(self.h, path)

    def load(self, path):
        lbm_load(self.h, path)

    def autotune(self, chunks=20, use_cache=True):
        return lbm_autotune(self.h, chunks, use_cache)

    def init_fields_device(self, rho, ux, uy, renormalise_mass=True, zero_staggered=False):
        lbm_init_fields_device(self.h, rho, ux, uy, renormalise_mass, zero_staggered)


class Batch:
    """Many cavities advanced together (one library batch handle)."""

    def __init__(self, nx, ny, re, u_lid=0.1, dtype="f64"):
        self.nx = [int(v) for v in nx]
        self.ny = [int(v) for v in ny]
        self.b = lbm_batch_create(self.nx, self.ny, re, u_lid, dtype)

    def close(self):
        if self.b:
            lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.nx)

    @property
    def info(self):
        return lbm_batch_info(self.b)

    def step(self, n=1):
        lbm_batch_step(self.b, n)
        return self

    def status(self, k):
        return lbm_batch_status(self.b, k)

    def set_threshold(self, r):
        lbm_batch_set_threshold(self.b, r)

    def set_active(self, k, active):
        lbm_batch_set_active(self.b, k, active)

    def mass(self, k):
        return lbm_batch_mass(self.b, k)

    def moments(self, k):
        return lbm_batch_moments(self.b, k, self.nx[k], self.ny[k])

    def get_populations(self, k):
        return lbm_batch_get_populations(self.b, k, self.nx[k], self.ny[k])

    def set_populations(self, k, f):
        lbm_batch_set_populations(self.b, k, f, self.nx[k], self.ny[k])

    def init_fields(self, k, rho=None, ux=None, uy=None, renormalise_mass=True,
                    zero_staggered=False):
        lbm_batch_init_fields(self.b, k, rho, ux, uy, self.nx[k], self.ny[k], renormalise_mass,
                              zero_staggered)

    def set_stream(self, stream):
        lbm_batch_set_stream(self.b, stream)

    def set_option(self, option, value):
        lbm_batch_set_option(self.b, option, value)

    def get_option(self, option):
        return lbm_batch_get_option(self.b, option)

    def autotune(self, chunks=2, use_cache=True):
        return lbm_batch_autotune(self.b, chunks, use_cache)

    def residuals(self):
        return lbm_batch_residuals(self.b, len(self.nx))

    def probe_config(self, xy, capacity):
        self.probe_npts = lbm_batch_probe_config(self.b, xy, capacity)

    def probe_read(self, k, max_records):
        return lbm_batch_probe_read(self.b, k, self.probe_npts, max_records)

    def probe_classify(self, component, window, steady_tol, periodic_tol, min_lag=1, max_lag=0):
        return lbm_batch_probe_classify(self.b, len(self.nx), self.probe_npts, component, window,
                                        steady_tol, periodic_tol, min_lag, max_lag)

    def cavity(self, k):
        return lbm_batch_cavity(self.b, k)

    def canvas(self, k, target, mask):
        lbm_batch_canvas(self.b, k, target, mask)


class Surrogate:
    """The warm-start network (one library surrogate handle)."""

    def __init__(self, max_batch=16):
        self.s = lbm_sur_create(max_batch)
        self.max_batch = max_batch

    def close(self):
        if self.s:
            lbm_sur_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self):
        return lbm_sur_num_params(self.s)

    def set_params(self, p):
        lbm_sur_set_params(self.s, p)

    def get_params(self, with_grads=False):
        return lbm_sur_get_params(self.s, with_grads)

    def set_stream(self, stream):
        lbm_sur_set_stream(self.s, stream)

    def forward(self, re, ar, out):
        lbm_sur_forward(self.s, re, ar, out)

    def train_step(self, re, ar, target, mask, lr, apply_update=True):
        return lbm_sur_train_step(self.s, re, ar, target, mask, lr, apply_update)

    def warm_start(self, cavity):
        lbm_sur_warm_start(self.s, cavity.h)

    def warm_start_batch(self, batch, k):
        lbm_sur_warm_start_batch(self.s, batch.b, k)


# ---------------------------------------------------------------- 3-D box
def lbm3d_create(nx, ny, nz, re, u_lid, dtype):
    h = _h()
    _check(_lib.lbm3d_create(int(nx), int(ny), int(nz), float(re), float(u_lid),
                             DTYPES.get(dtype, dtype), ct.byref(h)))
    return h


def lbm3d_destroy(h):
    _check(_lib.lbm3d_destroy(h))


def lbm3d_set_stream(h, stream):
    _check(_lib.lbm3d_set_stream(h, _stream_ptr(stream)))


def lbm3d_set_option(h, option, value):
    _check(_lib.lbm3d_set_option(h, int(option), int(value)))


def lbm3d_get_option(h, option):
    v = _i64()
    _check(_lib.lbm3d_get_option(h, int(option), ct.byref(v)))
    return v.value


def lbm3d_step(h, n):
    _check(_lib.lbm3d_step(h, int(n)))


def lbm3d_steps_done(h):
    v = _i64()
    _check(_lib.lbm3d_steps_done(h, ct.byref(v)))
    return v.value


def lbm3d_residual(h):
    r, t = ct.c_double(), _i64()
    _check(_lib.lbm3d_residual(h, ct.byref(r), ct.byref(t)))
    return r.value, t.value


def lbm3d_mass(h):
    m = ct.c_double()
    _check(_lib.lbm3d_mass(h, ct.byref(m)))
    return m.value


def lbm3d_moments(h, nx, ny, nz):
    out = [np.empty((nz, ny, nx)) for _ in range(4)]
    _check(_lib.lbm3d_moments(h, *[_ptr(a) for a in out]))
    return tuple(out)


def lbm3d_set_populations(h, f, nx, ny, nz):
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.shape != (19, nz, ny, nx):
        raise ValueError(f"populations must be [19, {nz}, {ny}, {nx}]")
    _check(_lib.lbm3d_set_populations(h, _ptr(f)))


def lbm3d_get_populations(h, nx, ny, nz):
    f = np.empty((19, nz, ny, nx))
    _check(_lib.lbm3d_get_populations(h, _ptr(f)))
    return f


def lbm3d_autotune(h, chunks=5):
    best, ms = ct.c_int(), ct.c_double()
    _check(_lib.lbm3d_autotune(h, int(chunks), ct.byref(best), ct.byref(ms)))
    return best.value, ms.value


class Cube:
    """A D3Q19 lid-driven box on the GPU (one library handle)."""

    def __init__(self, nx, ny, nz, re, u_lid=0.1, dtype="f64"):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.h = lbm3d_create(nx, ny, nz, re, u_lid, dtype)

    def close(self):
        if self.h:
            lbm3d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n):
        lbm3d_step(self.h, n)
        return self

    def moments(self):
        return lbm3d_moments(self.h, self.nx, self.ny, self.nz)

    def mass(self):
        return lbm3d_mass(self.h)

    def residual(self):
        return lbm3d_residual(self.h)

    def steps_done(self):
        return lbm3d_steps_done(self.h)

    def set_populations(self, f):
        lbm3d_set_populations(self.h, f, self.nx, self.ny, self.nz)

    def get_populations(self):
        return lbm3d_get_populations(self.h, self.nx, self.ny, self.nz)

    def set_option(self, option, value):
        lbm3d_set_option(self.h, option, value)

    def get_option(self, option):
        return lbm3d_get_option(self.h, option)

    def autotune(self, chunks=5):
        return lbm3d_autotune(self.h, chunks)
