"""Thin ctypes binding of ``libfluxlbm.so`` (see ``include/fluxlbm.h``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. PyTorch provides the device memory (one ``uint8`` tensor bound
to the context) and the stream (torch's current stream). There is no CPU
fallback: if the library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfluxlbm.so")

FLBM_OK = 0
FLBM_EINVAL = -1
FLBM_ENOINLET = -2
FLBM_ENOMEM = -3
FLBM_EHIP = -4
FLBM_EUNSTABLE = -5
FLBM_EINDEX = -6
FLBM_EBOUND = -7
FLBM_ESTATE = -8
FLBM_ESCRATCH = -9

FLBM_FP64, FLBM_FP32, FLBM_FP16DEV = 0, 1, 2
FLBM_BGK, FLBM_COLOUR, FLBM_MRT = 0, 1, 2
FLBM_Z_FLUX, FLBM_Z_PERIODIC, FLBM_Z_WALL = 0, 1, 2
FLBM_PULL_INT32, FLBM_PULL_HALF, FLBM_PULL_COMPACT, FLBM_PULL_RUN = 0, 1, 2, 3
PULL_HDR = 20  # int32 header entries per tile of the compact pull table

PRECISIONS = {"fp64": FLBM_FP64, "fp32": FLBM_FP32, "fp16dev": FLBM_FP16DEV}
MODELS = {"bgk": FLBM_BGK, "colour": FLBM_COLOUR, "mrt": FLBM_MRT}


class FlbmError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: status {status}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


class flbm_controller_params(ctypes.Structure):
    _fields_ = [
        ("geometry", ctypes.c_float * 15), ("margin", ctypes.c_float),
        ("drho_ref", ctypes.c_double), ("gain", ctypes.c_double), ("trust0", ctypes.c_double), ("release_tol", ctypes.c_double),
        ("trust_decisions", ctypes.c_int32), ("relative", ctypes.c_int32),
        ("stall_decisions", ctypes.c_int32), ("period", ctypes.c_int32),
    ]


class flbm_schedule(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("order", ctypes.c_int32), ("tiles_per_item", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("occupancy", ctypes.c_int32)]


FLBM_ORDER_SAMPLE, FLBM_ORDER_INTERLEAVE, FLBM_ORDER_LARGEST = 0, 1, 2


class flbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
        ("z_mode", ctypes.c_int32), ("reservoir_layers", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("model", ctypes.c_int32),
        ("watchdog_every", ctypes.c_int32),
        ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
        ("q_target", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("phi_solid", ctypes.c_double), ("umax_limit", ctypes.c_double),
    ]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64P = ctypes.POINTER(ctypes.c_int64)
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)

# name -> argtypes (all return int32 status unless listed in _RESTYPES)
_SIGS = {
    "flbm_default_params": [ctypes.POINTER(flbm_params)],
    "flbm_create": [_P, ctypes.POINTER(flbm_params), _P, ctypes.POINTER(_P)],
    "flbm_destroy": [_P],
    "flbm_device_bytes": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "flbm_bind_device_memory": [_P, _P, ctypes.c_size_t],
    "flbm_num_sites": [_P, _I64P, _I64P, _I64P],
    "flbm_get_site_coords": [_P, _P],
    "flbm_init_equilibrium": [_P, _D, _D, _D, _D],
    "flbm_set_target_flux": [_P, _D],
    "flbm_set_outlet_density": [_P, _D],
    "flbm_step": [_P, _I32],
    "flbm_sync": [_P],
    "flbm_get_boundary": [_P, _DP, _DP, _DP, _DP],
    "flbm_get_history": [_P, _P, _I32],
    "flbm_history_capacity": [_P, ctypes.POINTER(_I32)],
    "flbm_step_count": [_P, _I64P],
    "flbm_read_fields": [_P, _P, _P, _P, _P],
    "flbm_read_distributions": [_P, _P],
    "flbm_write_distributions": [_P, _P],
    "flbm_init_colour": [_P, _P, _P],
    "flbm_read_colour": [_P, _P, _P],
    "flbm_write_colour": [_P, _P, _P],
    "flbm_read_phase": [_P, _P],
    "flbm_get_pull_table": [_P, _P],
    "flbm_set_pull_format": [_P, _I32, _I32, _I32],
    "flbm_pull_format_info": [_P, ctypes.POINTER(_I32), _I64P, _I64P, _I64P],
    "flbm_get_compact_pull": [_P, _P, _P, _P, _P],
    "flbm_pull_run_info": [_P, _I64P, _I64P],
    "flbm_get_pull_runs": [_P, _P, _P],
    "flbm_state_bytes": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "flbm_save_state": [_P, _P, ctypes.c_size_t],
    "flbm_load_state": [_P, _P, ctypes.c_size_t],
    "flbm_debug_set_collision": [_P, _I32],
    "flbm_get_observables": [_P, _DP, _DP, ctypes.POINTER(_I32)],
    "flbm_state_observables_noalloc": [_P, _I32, ctypes.c_int64, ctypes.c_int64, _D, _P, _DP, _DP,
                                       ctypes.POINTER(_I32)],
    "flbm_device_layout": [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _I64P],
    "flbm_profile_kernels": [_P, _I32, _DP, _DP],
    "flbm_copy_kernel": [_P, _P, ctypes.c_size_t, _P],
    "flbm_mlp_create": [_I32, _P, ctypes.POINTER(_P)],
    "flbm_mlp_destroy": [_P],
    "flbm_mlp_num_params": [ctypes.POINTER(_I32)],
    "flbm_mlp_set_params": [_P, _P, _I32],
    "flbm_mlp_get_params": [_P, _P, _I32],
    "flbm_mlp_forward": [_P, _P, _P, _I32],
    "flbm_mlp_gradients": [_P, _P, _P, _I32, _P, _P],
    "flbm_mlp_train_step": [_P, _P, _P, _I32, ctypes.c_float, _P],
    "flbm_gemm_bf16": [_P, ctypes.c_int64, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int64, _P,
                       ctypes.c_int64, _I32, _I32, _I32, _P],
    "flbm_set_controller": [_P, _P, _P],
    "flbm_controller_state": [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), _DP, _I64P],
    "flbm_controller_trace": [_P, _I32, _P, _P],
    "flbm_set_inlet_density_override": [_P, _DP, _D],
    "flbm_batch_create": [_I32, _P, ctypes.POINTER(_P)],
    "flbm_batch_destroy": [_P],
    "flbm_batch_set_schedule": [_P, _P],
    "flbm_batch_get_schedule": [_P, _P],
    "flbm_batch_step": [_P, _I32],
    "flbm_batch_sync": [_P, ctypes.POINTER(_I32)],
    "flbm_batch_time": [_P, _I32, _DP],
    "flbm_batch_autotune": [_P, ctypes.c_char_p, _I32, _P, _DP],
    "flbm_batch_last_error": [_P],
    "flbm_status_string": [_I32],
    "flbm_last_error": [_P],
}
_RESTYPES = {"flbm_status_string": ctypes.c_char_p, "flbm_last_error": ctypes.c_char_p,
             "flbm_batch_last_error": ctypes.c_char_p}

_lib = None


def load_library(path: str | None = None):
    """Load libfluxlbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library {path} is missing: build it with `python -m paper_1806_10589_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, argtypes in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = _RESTYPES.get(name, _I32)
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _check(rc: int, where: str, ctx=None):
    if rc != FLBM_OK:
        lib = load_library()
        detail = lib.flbm_status_string(rc).decode()
        if ctx:
            extra = lib.flbm_last_error(ctx)
            if extra:
                detail += ": " + extra.decode()
        raise FlbmError(rc, where, detail)


# ------------------------------------------------------------------ C-ABI names

def flbm_default_params() -> flbm_params:
    p = flbm_params()
    _check(load_library().flbm_default_params(ctypes.byref(p)), "flbm_default_params")
    return p


def flbm_create(mask: np.ndarray, params: flbm_params, stream: int | None = None):
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    ctx = _P()
    _check(load_library().flbm_create(mask.ctypes.data, ctypes.byref(params), stream or None,
                                      ctypes.byref(ctx)), "flbm_create")
    return ctx


def flbm_destroy(ctx) -> None:
    _check(load_library().flbm_destroy(ctx), "flbm_destroy")


def flbm_device_bytes(ctx) -> int:
    v = ctypes.c_size_t()
    _check(load_library().flbm_device_bytes(ctx, ctypes.byref(v)), "flbm_device_bytes", ctx)
    return int(v.value)


def flbm_bind_device_memory(ctx, dev_ptr: int, nbytes: int) -> None:
    _check(load_library().flbm_bind_device_memory(ctx, dev_ptr, nbytes), "flbm_bind_device_memory", ctx)


def flbm_num_sites(ctx):
    n, a, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().flbm_num_sites(ctx, ctypes.byref(n), ctypes.byref(a), ctypes.byref(b)),
           "flbm_num_sites", ctx)
    return int(n.value), int(a.value), int(b.value)


def flbm_get_site_coords(ctx, n_sites: int) -> np.ndarray:
    out = np.empty((n_sites, 3), np.int32)
    _check(load_library().flbm_get_site_coords(ctx, out.ctypes.data), "flbm_get_site_coords", ctx)
    return out


def flbm_init_equilibrium(ctx, rho=1.0, ux=0.0, uy=0.0, uz=0.0) -> None:
    _check(load_library().flbm_init_equilibrium(ctx, rho, ux, uy, uz), "flbm_init_equilibrium", ctx)


def flbm_set_target_flux(ctx, q: float) -> None:
    _check(load_library().flbm_set_target_flux(ctx, q), "flbm_set_target_flux", ctx)


def flbm_set_outlet_density(ctx, rho: float) -> None:
    _check(load_library().flbm_set_outlet_density(ctx, rho), "flbm_set_outlet_density", ctx)


def flbm_step(ctx, n: int) -> None:
    _check(load_library().flbm_step(ctx, int(n)), "flbm_step", ctx)


def flbm_sync(ctx) -> int:
    """Returns the status (FLBM_OK or FLBM_EUNSTABLE); raises on other errors."""
    rc = load_library().flbm_sync(ctx)
    if rc not in (FLBM_OK, FLBM_EUNSTABLE):
        _check(rc, "flbm_sync", ctx)
    return rc


def flbm_get_boundary(ctx):
    v = [_D() for _ in range(4)]
    _check(load_library().flbm_get_boundary(ctx, *[ctypes.byref(x) for x in v]), "flbm_get_boundary", ctx)
    return tuple(float(x.value) for x in v)


def flbm_get_history(ctx, n: int) -> np.ndarray:
    """(n, 7): rho_in, Q_in, Q_out, mass, max|u|, sum N_A, sum N_B."""
    out = np.empty((n, 7), np.float64)
    _check(load_library().flbm_get_history(ctx, out.ctypes.data, int(n)), "flbm_get_history", ctx)
    return out


def flbm_history_capacity(ctx) -> int:
    v = _I32()
    _check(load_library().flbm_history_capacity(ctx, ctypes.byref(v)), "flbm_history_capacity", ctx)
    return int(v.value)


def flbm_step_count(ctx) -> int:
    v = ctypes.c_int64()
    _check(load_library().flbm_step_count(ctx, ctypes.byref(v)), "flbm_step_count", ctx)
    return int(v.value)


def flbm_read_fields(ctx, n_sites: int):
    arrs = [np.empty(n_sites, np.float64) for _ in range(4)]
    _check(load_library().flbm_read_fields(ctx, *[a.ctypes.data for a in arrs]), "flbm_read_fields", ctx)
    return tuple(arrs)


def flbm_read_distributions(ctx, n_sites: int) -> np.ndarray:
    out = np.empty((19, n_sites), np.float64)
    _check(load_library().flbm_read_distributions(ctx, out.ctypes.data), "flbm_read_distributions", ctx)
    return out


def flbm_write_distributions(ctx, f: np.ndarray) -> None:
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(load_library().flbm_write_distributions(ctx, f.ctypes.data), "flbm_write_distributions", ctx)


def flbm_init_colour(ctx, na: np.ndarray, nb: np.ndarray) -> None:
    na = np.ascontiguousarray(na, dtype=np.float64)
    nb = np.ascontiguousarray(nb, dtype=np.float64)
    _check(load_library().flbm_init_colour(ctx, na.ctypes.data, nb.ctypes.data), "flbm_init_colour", ctx)


def flbm_read_colour(ctx, n_sites: int):
    A = np.empty((7, n_sites), np.float64)
    B = np.empty((7, n_sites), np.float64)
    _check(load_library().flbm_read_colour(ctx, A.ctypes.data, B.ctypes.data), "flbm_read_colour", ctx)
    return A, B


def flbm_write_colour(ctx, A: np.ndarray, B: np.ndarray) -> None:
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    _check(load_library().flbm_write_colour(ctx, A.ctypes.data, B.ctypes.data), "flbm_write_colour", ctx)


def flbm_read_phase(ctx, n_sites: int) -> np.ndarray:
    out = np.empty(n_sites, np.float64)
    _check(load_library().flbm_read_phase(ctx, out.ctypes.data), "flbm_read_phase", ctx)
    return out


def flbm_get_pull_table(ctx, n_sites: int) -> np.ndarray:
    out = np.empty((18, n_sites), np.int32)
    _check(load_library().flbm_get_pull_table(ctx, out.ctypes.data), "flbm_get_pull_table", ctx)
    return out


def flbm_set_pull_format(ctx, fmt: int, limit16: int = 0, limit8: int = 0) -> None:
    _check(load_library().flbm_set_pull_format(ctx, int(fmt), int(limit16), int(limit8)), "flbm_set_pull_format",
           ctx)


def flbm_pull_format_info(ctx):
    """(format, tiles with 8-bit codes, tiles with 16-bit codes, tiles)."""
    f, t8, t16, t = _I32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().flbm_pull_format_info(ctx, ctypes.byref(f), ctypes.byref(t8), ctypes.byref(t16),
                                                ctypes.byref(t)), "flbm_pull_format_info", ctx)
    return int(f.value), int(t8.value), int(t16.value), int(t.value)


def flbm_get_compact_pull(ctx, n_pad: int, tiles: int):
    """Host copy of the compact pull table: 16-bit codes uint32 [9][n_pad],
    8-bit codes uint32 [4][n_pad] and uint16 [n_pad], header int32
    [tiles][PULL_HDR]."""
    codes16 = np.empty((9, n_pad), np.uint32)
    codes8 = np.empty((4, n_pad), np.uint32)
    tail = np.empty(n_pad, np.uint16)
    hdr = np.empty((tiles, PULL_HDR), np.int32)
    _check(load_library().flbm_get_compact_pull(ctx, codes16.ctypes.data, codes8.ctypes.data, tail.ctypes.data,
                                                hdr.ctypes.data), "flbm_get_compact_pull", ctx)
    return codes16, codes8, tail, hdr


def flbm_pull_run_info(ctx):
    """(8-bit tiles with run codes, their waves listing more than 256 codes)."""
    t, w = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().flbm_pull_run_info(ctx, ctypes.byref(t), ctypes.byref(w)), "flbm_pull_run_info", ctx)
    return int(t.value), int(w.value)


def flbm_get_pull_runs(ctx, n_pad: int):
    """Host copy of the run codes: uint32 [n_pad][2] (mask, list bytes
    4l..4l+3) and uint32 [n_pad] (list bytes 256+4l..256+4l+3)."""
    runs = np.empty((n_pad, 2), np.uint32)
    runs_hi = np.empty(n_pad, np.uint32)
    _check(load_library().flbm_get_pull_runs(ctx, runs.ctypes.data, runs_hi.ctypes.data), "flbm_get_pull_runs", ctx)
    return runs, runs_hi


def flbm_state_bytes(ctx) -> int:
    v = ctypes.c_size_t()
    _check(load_library().flbm_state_bytes(ctx, ctypes.byref(v)), "flbm_state_bytes", ctx)
    return int(v.value)


def flbm_save_state(ctx) -> bytes:
    n = flbm_state_bytes(ctx)
    buf = ctypes.create_string_buffer(n)
    _check(load_library().flbm_save_state(ctx, buf, n), "flbm_save_state", ctx)
    return buf.raw


def flbm_load_state(ctx, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(load_library().flbm_load_state(ctx, buf, len(blob)), "flbm_load_state", ctx)


def flbm_debug_set_collision(ctx, enabled: bool) -> None:
    _check(load_library().flbm_debug_set_collision(ctx, int(bool(enabled))), "flbm_debug_set_collision", ctx)


def flbm_get_observables(ctx):
    m, u, b = _D(), _D(), _I32()
    _check(load_library().flbm_get_observables(ctx, ctypes.byref(m), ctypes.byref(u), ctypes.byref(b)),
           "flbm_get_observables", ctx)
    return float(m.value), float(u.value), int(b.value)


def flbm_state_observables_noalloc(f_dev: int, precision: int, n_sites: int, n_pad: int, rho0: float,
                                   stream: int | None):
    """(mass, max |u|, non-finite flag) of a device state [19][n_pad] the
    caller holds, by the allocation-free entry point."""
    m, u, b = _D(), _D(), _I32()
    _check(load_library().flbm_state_observables_noalloc(f_dev, precision, n_sites, n_pad, rho0, stream,
                                                         ctypes.byref(m), ctypes.byref(u), ctypes.byref(b)),
           "flbm_state_observables_noalloc")
    return float(m.value), float(u.value), int(b.value)


def flbm_device_layout(ctx):
    f, nb, npad = _P(), _P(), ctypes.c_int64()
    _check(load_library().flbm_device_layout(ctx, ctypes.byref(f), ctypes.byref(nb), ctypes.byref(npad)),
           "flbm_device_layout", ctx)
    return f.value, nb.value, int(npad.value)


def flbm_profile_kernels(ctx, n: int):
    a, b = _D(), _D()
    _check(load_library().flbm_profile_kernels(ctx, int(n), ctypes.byref(a), ctypes.byref(b)),
           "flbm_profile_kernels", ctx)
    return float(a.value), float(b.value)


def flbm_copy_kernel(src: int, dst: int, nbytes: int, stream: int | None = None) -> None:
    _check(load_library().flbm_copy_kernel(src, dst, nbytes, stream or None), "flbm_copy_kernel")


def flbm_mlp_create(max_batch: int, stream: int | None = None):
    out = _P()
    _check(load_library().flbm_mlp_create(int(max_batch), stream or None, ctypes.byref(out)), "flbm_mlp_create")
    return out.value


def flbm_mlp_destroy(m) -> None:
    _check(load_library().flbm_mlp_destroy(m), "flbm_mlp_destroy")


def flbm_mlp_num_params() -> int:
    n = _I32()
    _check(load_library().flbm_mlp_num_params(ctypes.byref(n)), "flbm_mlp_num_params")
    return int(n.value)


def flbm_mlp_set_params(m, params: np.ndarray) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(load_library().flbm_mlp_set_params(m, p.ctypes.data, p.size), "flbm_mlp_set_params")


def flbm_mlp_get_params(m) -> np.ndarray:
    p = np.empty(flbm_mlp_num_params(), dtype=np.float32)
    _check(load_library().flbm_mlp_get_params(m, p.ctypes.data, p.size), "flbm_mlp_get_params")
    return p


def flbm_mlp_forward(m, dev_x: int, dev_y: int, batch: int) -> None:
    _check(load_library().flbm_mlp_forward(m, dev_x, dev_y, int(batch)), "flbm_mlp_forward")


def flbm_mlp_gradients(m, dev_x: int, dev_t: int, batch: int):
    g = np.empty(flbm_mlp_num_params(), dtype=np.float32)
    loss = np.empty(1, dtype=np.float32)
    _check(load_library().flbm_mlp_gradients(m, dev_x, dev_t, int(batch), g.ctypes.data, loss.ctypes.data),
           "flbm_mlp_gradients")
    return g, float(loss[0])


def flbm_mlp_train_step(m, dev_x: int, dev_t: int, batch: int, lr: float, want_loss: bool = False):
    loss = np.empty(1, dtype=np.float32)
    _check(load_library().flbm_mlp_train_step(m, dev_x, dev_t, int(batch), float(lr),
                                              loss.ctypes.data if want_loss else None), "flbm_mlp_train_step")
    return float(loss[0]) if want_loss else None


def flbm_gemm_bf16(a: int, a_rs: int, a_cs: int, b: int, b_rs: int, b_cs: int, c: int, c_rs: int,
                   m: int, n: int, k: int, stream: int | None = None) -> None:
    _check(load_library().flbm_gemm_bf16(a, a_rs, a_cs, b, b_rs, b_cs, c, c_rs, m, n, k, stream or None),
           "flbm_gemm_bf16")


def flbm_set_controller(ctx, net, params: flbm_controller_params | None) -> None:
    _check(load_library().flbm_set_controller(ctx, net, ctypes.byref(params) if params is not None else None),
           "flbm_set_controller", ctx)


def flbm_controller_state(ctx):
    a, r, d, n = _I32(), _I32(), _D(), ctypes.c_int64()
    _check(load_library().flbm_controller_state(ctx, ctypes.byref(a), ctypes.byref(r), ctypes.byref(d),
                                                ctypes.byref(n)), "flbm_controller_state", ctx)
    return bool(a.value), bool(r.value), float(d.value), int(n.value)


def flbm_set_inlet_density_override(ctx, rho_in, trust: float = 1.0) -> None:
    if rho_in is None:
        _check(load_library().flbm_set_inlet_density_override(ctx, None, 0.0), "flbm_set_inlet_density_override",
               ctx)
    else:
        r = _D(float(rho_in))
        _check(load_library().flbm_set_inlet_density_override(ctx, ctypes.byref(r), float(trust)),
               "flbm_set_inlet_density_override", ctx)


def flbm_controller_trace(ctx, n: int):
    x = np.empty((int(n), 32), dtype=np.float32)
    aux = np.empty((int(n), 4), dtype=np.float64)
    _check(load_library().flbm_controller_trace(ctx, int(n), x.ctypes.data, aux.ctypes.data),
           "flbm_controller_trace", ctx)
    return x, aux


def _bcheck(rc: int, where: str, b):
    if rc != FLBM_OK:
        lib = load_library()
        detail = lib.flbm_status_string(rc).decode()
        extra = lib.flbm_batch_last_error(b) if b else b""
        if extra:
            detail += ": " + extra.decode()
        raise FlbmError(rc, where, detail)


def flbm_batch_create(ctxs):
    arr = (_P * len(ctxs))(*ctxs)
    out = _P()
    _bcheck(load_library().flbm_batch_create(len(ctxs), arr, ctypes.byref(out)), "flbm_batch_create", None)
    return out.value


def flbm_batch_destroy(b) -> None:
    _bcheck(load_library().flbm_batch_destroy(b), "flbm_batch_destroy", None)


def flbm_batch_set_schedule(b, sched: flbm_schedule) -> None:
    _bcheck(load_library().flbm_batch_set_schedule(b, ctypes.byref(sched)), "flbm_batch_set_schedule", b)


def flbm_batch_get_schedule(b) -> flbm_schedule:
    s = flbm_schedule()
    _bcheck(load_library().flbm_batch_get_schedule(b, ctypes.byref(s)), "flbm_batch_get_schedule", b)
    return s


def flbm_batch_step(b, n: int) -> None:
    _bcheck(load_library().flbm_batch_step(b, int(n)), "flbm_batch_step", b)


def flbm_batch_sync(b):
    i = _I32(-1)
    rc = load_library().flbm_batch_sync(b, ctypes.byref(i))
    return rc, int(i.value)


def flbm_batch_time(b, n: int) -> float:
    ms = _D()
    _bcheck(load_library().flbm_batch_time(b, int(n), ctypes.byref(ms)), "flbm_batch_time", b)
    return float(ms.value)


def flbm_batch_autotune(b, cache_path: str | None, trial_steps: int):
    s, ms = flbm_schedule(), _D()
    _bcheck(load_library().flbm_batch_autotune(b, cache_path.encode() if cache_path else None, int(trial_steps),
                                               ctypes.byref(s), ctypes.byref(ms)), "flbm_batch_autotune", b)
    return s, float(ms.value)


# ------------------------------------------------------------------ convenience

class Mlp:
    """The controller network on ``device``, working on torch's current
    stream; inputs and targets are torch FP32 device tensors."""

    def __init__(self, max_batch: int, device: str = "cuda:0"):
        import torch

        self.device = torch.device(device)
        self._torch = torch
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.handle = flbm_mlp_create(max_batch, self.stream.cuda_stream)
        self.max_batch = int(max_batch)
        self.n_params = flbm_mlp_num_params()

    def close(self):
        if getattr(self, "handle", None):
            flbm_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, t, shape):
        t = t.to(self.device, self._torch.float32).contiguous()
        if tuple(t.shape) != shape:
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return t

    def set_params(self, p: np.ndarray):
        flbm_mlp_set_params(self.handle, p)

    def get_params(self) -> np.ndarray:
        return flbm_mlp_get_params(self.handle)

    def forward(self, x):
        b = int(x.shape[0])
        x = self._dev(x, (b, 32))
        y = self._torch.empty(b, dtype=self._torch.float32, device=self.device)
        flbm_mlp_forward(self.handle, x.data_ptr(), y.data_ptr(), b)
        return y

    def gradients(self, x, t):
        b = int(x.shape[0])
        x, t = self._dev(x, (b, 32)), self._dev(t, (b,))
        return flbm_mlp_gradients(self.handle, x.data_ptr(), t.data_ptr(), b)

    def train_step(self, x, t, lr, want_loss=False):
        b = int(x.shape[0])
        x, t = self._dev(x, (b, 32)), self._dev(t, (b,))
        return flbm_mlp_train_step(self.handle, x.data_ptr(), t.data_ptr(), b, lr, want_loss)


class Lattice:
    """A context whose device memory is one torch ``uint8`` tensor and whose
    stream is torch's current stream on ``device``.

    Parameters mirror ``flbm_params``; the mask is ``uint8 (nz, ny, nx)``.
    """

    def __init__(self, mask: np.ndarray, *, tau: float = 0.8, q_target: float = 0.0,
                 rho_out: float = 1.0, rho0: float = 1.0, precision: str = "fp32",
                 model: str = "bgk", periodic_x: bool = True, periodic_y: bool = True,
                 z_mode: int = FLBM_Z_FLUX, reservoir_layers: int = 0,
                 watchdog_every: int = 1000, umax_limit: float = 0.1, alpha: float | None = None,
                 beta: float | None = None, phi_solid: float | None = None,
                 device: str = "cuda:0"):
        import torch

        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.ndim != 3:
            raise ValueError("mask must be (nz, ny, nx)")
        p = flbm_default_params()
        p.nz, p.ny, p.nx = mask.shape
        p.periodic_x, p.periodic_y = int(periodic_x), int(periodic_y)
        p.z_mode = int(z_mode)
        p.reservoir_layers = int(reservoir_layers)
        p.precision = PRECISIONS[precision]
        p.model = MODELS[model]
        p.watchdog_every = int(watchdog_every)
        p.tau, p.rho0, p.q_target, p.rho_out = float(tau), float(rho0), float(q_target), float(rho_out)
        p.umax_limit = float(umax_limit)
        if alpha is not None:
            p.alpha = float(alpha)
        if beta is not None:
            p.beta = float(beta)
        if phi_solid is not None:
            p.phi_solid = float(phi_solid)
        self.params = p
        self.device = torch.device(device)
        self._torch = torch
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.ctx = flbm_create(mask, p, self.stream.cuda_stream)
            try:
                self.n_sites, self.a_in, self.a_out = flbm_num_sites(self.ctx)
                nbytes = flbm_device_bytes(self.ctx)
                self._mem = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
                base = self._mem.data_ptr()
                aligned = (base + 255) // 256 * 256
                flbm_bind_device_memory(self.ctx, aligned, nbytes)
            except Exception:
                flbm_destroy(self.ctx)
                self.ctx = None
                raise
        self.device_bytes = nbytes

    def close(self):
        if getattr(self, "ctx", None):
            flbm_destroy(self.ctx)
            self.ctx = None
            self._mem = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # thin forwards -------------------------------------------------------------
    def coords(self) -> np.ndarray:
        return flbm_get_site_coords(self.ctx, self.n_sites)

    def init_equilibrium(self, rho=1.0, ux=0.0, uy=0.0, uz=0.0):
        flbm_init_equilibrium(self.ctx, rho, ux, uy, uz)

    def set_target_flux(self, q):
        flbm_set_target_flux(self.ctx, q)

    def set_outlet_density(self, rho):
        flbm_set_outlet_density(self.ctx, rho)

    def step(self, n=1):
        flbm_step(self.ctx, n)

    def sync(self) -> int:
        return flbm_sync(self.ctx)

    def boundary(self):
        return flbm_get_boundary(self.ctx)

    def history(self, n):
        return flbm_get_history(self.ctx, n)

    @property
    def step_count(self):
        return flbm_step_count(self.ctx)

    def fields(self):
        return flbm_read_fields(self.ctx, self.n_sites)

    def read_distributions(self):
        return flbm_read_distributions(self.ctx, self.n_sites)

    def write_distributions(self, f):
        flbm_write_distributions(self.ctx, f)

    def init_colour(self, na, nb):
        flbm_init_colour(self.ctx, na, nb)

    def read_colour(self):
        return flbm_read_colour(self.ctx, self.n_sites)

    def write_colour(self, A, B):
        flbm_write_colour(self.ctx, A, B)

    def phase(self):
        return flbm_read_phase(self.ctx, self.n_sites)

    def pull_table(self):
        return flbm_get_pull_table(self.ctx, self.n_sites)

    def set_pull_format(self, fmt: int, limit16: int = 0, limit8: int = 0):
        flbm_set_pull_format(self.ctx, fmt, limit16, limit8)

    def pull_format(self):
        """(format, tiles with 8-bit codes, tiles with 16-bit codes, tiles)."""
        return flbm_pull_format_info(self.ctx)

    def pull_runs(self):
        """(8-bit tiles with run codes, their waves listing more than 256 codes)."""
        return flbm_pull_run_info(self.ctx)

    def compact_pull(self):
        _, _, _, tiles = flbm_pull_format_info(self.ctx)
        _, _, n_pad = flbm_device_layout(self.ctx)
        return flbm_get_compact_pull(self.ctx, n_pad, tiles)

    def save_state(self) -> bytes:
        return flbm_save_state(self.ctx)

    def load_state(self, blob: bytes):
        flbm_load_state(self.ctx, blob)

    def set_collision(self, enabled: bool):
        flbm_debug_set_collision(self.ctx, enabled)

    def observables(self):
        return flbm_get_observables(self.ctx)

    def profile_kernels(self, n):
        return flbm_profile_kernels(self.ctx, n)

    def layout(self):
        return flbm_device_layout(self.ctx)

    def set_controller(self, net: "Mlp | None", geometry=None, *, drho_ref=1e-3, gain=1.0, trust0=0.5,
                       release_tol=1e-3, trust_decisions=20000, relative=False, stall_decisions=0, period=1,
                       margin=0.0):
        if net is None:
            flbm_set_controller(self.ctx, None, None)
            self._ctrl_net = None
            return
        p = flbm_controller_params()
        g = np.zeros(15, dtype=np.float32) if geometry is None else np.asarray(geometry, np.float32)
        if g.shape != (15,):
            raise ValueError("geometry must hold 15 features")
        for i in range(15):
            p.geometry[i] = float(g[i])
        p.drho_ref = float(drho_ref)
        p.relative, p.stall_decisions, p.period = int(bool(relative)), int(stall_decisions), int(period)
        p.margin = float(margin)
        p.gain, p.trust0, p.release_tol = float(gain), float(trust0), float(release_tol)
        p.trust_decisions = int(trust_decisions)
        flbm_set_controller(self.ctx, net.handle, p)
        self._ctrl_net = net  # the network must outlive the attachment

    def controller_state(self):
        return flbm_controller_state(self.ctx)

    def controller_trace(self, n):
        return flbm_controller_trace(self.ctx, n)

    def set_inlet_density_override(self, rho_in, trust=1.0):
        flbm_set_inlet_density_override(self.ctx, rho_in, trust)


class Batch:
    """Many ``Lattice`` objects (same device, stream, precision and model)
    stepped together by one launch per step."""

    def __init__(self, lattices):
        self.lattices = list(lattices)
        self.handle = flbm_batch_create([l.ctx for l in self.lattices])

    def close(self):
        if getattr(self, "handle", None):
            flbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        flbm_batch_step(self.handle, n)

    def sync(self):
        return flbm_batch_sync(self.handle)

    def time(self, n):
        return flbm_batch_time(self.handle, n)

    @property
    def schedule(self):
        s = flbm_batch_get_schedule(self.handle)
        return dict(grid=s.grid, order=s.order, tiles_per_item=s.tiles_per_item, chunk=s.chunk,
                    occupancy=s.occupancy)

    def set_schedule(self, grid=0, order=FLBM_ORDER_INTERLEAVE, tiles_per_item=4, chunk=64, occupancy=0):
        flbm_batch_set_schedule(self.handle, flbm_schedule(grid, order, tiles_per_item, chunk, occupancy))

    def autotune(self, cache_path=None, trial_steps=5):
        s, ms = flbm_batch_autotune(self.handle, cache_path, trial_steps)
        return dict(grid=s.grid, order=s.order, tiles_per_item=s.tiles_per_item, chunk=s.chunk,
                    occupancy=s.occupancy), ms

