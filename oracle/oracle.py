"""ctypes wrapper of the C oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE: used by the tests, the smoke check and the CPU baseline
of the benchmark only. Builds ``liboracle.so`` with gcc on first use.

Dense layout: distributions are numpy arrays of shape ``(nz, ny, nx, 19)``;
masks are ``uint8`` arrays of shape ``(nz, ny, nx)`` with 1 = solid.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["lbm_oracle.c"]
_lock = threading.Lock()
_lib = None

Z_FLUX, Z_PERIODIC, Z_WALL = 0, 1, 2

_d = ctypes.c_double
_i = ctypes.c_int
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_create.restype = _p
        lib.orc_create.argtypes = [_i, _i, _i, _p, _i, _i, _i, _d, _d, _d, _d]
        lib.orc_destroy.argtypes = [_p]
        lib.orc_set_collision.argtypes = [_p, _i]
        lib.orc_set_target_flux.argtypes = [_p, _d]
        lib.orc_set_outlet_density.argtypes = [_p, _d]
        lib.orc_set_inlet_offset.argtypes = [_p, _d]
        lib.orc_set_mrt.argtypes = [_p, _i]
        lib.orc_plain_inlet_density.argtypes = [_p]
        lib.orc_plain_inlet_density.restype = _d
        lib.orc_step_count.argtypes = [_p]
        lib.orc_step_count.restype = ctypes.c_long
        lib.orc_inlet_area.argtypes = [_p]
        lib.orc_outlet_area.argtypes = [_p]
        lib.orc_set_threads.argtypes = [_i]
        lib.orc_max_threads.restype = _i
        lib.orc_init_equilibrium.argtypes = [_p, _d, _d, _d, _d]
        lib.orc_set_f.argtypes = [_p, _p]
        lib.orc_get_f.argtypes = [_p, _p]
        lib.orc_fields.argtypes = [_p, _p, _p, _p, _p]
        lib.orc_step.argtypes = [_p, _i, _p]
        lib.orc_step.restype = _i
        lib.orc_velocity_set.argtypes = [_p, _p, _p, _p, _p]
        lib.orc_equilibrium.argtypes = [_d, _d, _d, _d, _d, _p]
        lib.orc_inlet_bc_site.argtypes = [_p, _d, _d]
        lib.orc_inlet_bc_site.restype = _d
        lib.orc_outlet_bc_site.argtypes = [_p, _d, _d]
        lib.orc_outlet_bc_site.restype = _d
        lib.orc_mrt_matrix.argtypes = [_p]
        lib.orc_mrt_collide_site.argtypes = [_p, _d, _d, _d, _d, _d, _d]
        lib.orc_mrt_collide_site_rates.argtypes = [_p, _d, _p, _d, _d, _d, _d]
        lib.orc_colour_create.restype = _p
        lib.orc_colour_create.argtypes = [_i, _i, _i, _p, _i, _i, _i, _d, _d, _d, _d, _d, _d, _d]
        lib.orc_colour_destroy.argtypes = [_p]
        lib.orc_colour_init.argtypes = [_p, _p, _p]
        lib.orc_colour_set_state.argtypes = [_p, _p, _p, _p]
        lib.orc_colour_get_state.argtypes = [_p, _p, _p, _p]
        lib.orc_colour_step.argtypes = [_p, _i, _p]
        lib.orc_colour_step.restype = _i
        lib.orc_colour_fields.argtypes = [_p, _p, _p, _p, _p, _p]
        lib.orc_colour_set_collision.argtypes = [_p, _i]
        lib.orc_colour_gradient.argtypes = [_p, _p, _p]
        _lib = lib
        return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def velocity_set():
    """(cx, cy, cz, w, opp) of the oracle's D3Q19 numbering."""
    lib = _load()
    cx = np.zeros(19, np.int32)
    cy = np.zeros(19, np.int32)
    cz = np.zeros(19, np.int32)
    w = np.zeros(19, np.float64)
    opp = np.zeros(19, np.int32)
    lib.orc_velocity_set(_ptr(cx), _ptr(cy), _ptr(cz), _ptr(w), _ptr(opp))
    return cx, cy, cz, w, opp


def equilibrium(rho, ux, uy, uz, rho0=1.0) -> np.ndarray:
    lib = _load()
    out = np.zeros(19, np.float64)
    lib.orc_equilibrium(float(rho), float(rho0), float(ux), float(uy), float(uz), _ptr(out))
    return out


def inlet_bc_site(f: np.ndarray, rho: float, rho0: float = 1.0):
    """Apply the inlet pressure condition to one site's 19 values; returns (f, u_z)."""
    lib = _load()
    g = np.ascontiguousarray(f, dtype=np.float64).copy()
    uz = lib.orc_inlet_bc_site(_ptr(g), float(rho), float(rho0))
    return g, uz


def outlet_bc_site(f: np.ndarray, rho: float, rho0: float = 1.0):
    lib = _load()
    g = np.ascontiguousarray(f, dtype=np.float64).copy()
    uz = lib.orc_outlet_bc_site(_ptr(g), float(rho), float(rho0))
    return g, uz


def mrt_matrix() -> np.ndarray:
    """The 19x19 moment matrix M (rows: moments in Appendix A's order)."""
    out = np.zeros((19, 19), np.float64)
    _load().orc_mrt_matrix(_ptr(out))
    return out


def mrt_collide_site(f, tau, alpha=0.0, grad=(0.0, 0.0, 0.0), rho0=1.0) -> np.ndarray:
    """One site's MRT collision with the colour stress of gradient `grad`."""
    g = np.ascontiguousarray(f, dtype=np.float64).copy()
    _load().orc_mrt_collide_site(_ptr(g), float(rho0), float(tau), float(alpha), *map(float, grad))
    return g


def mrt_collide_site_rates(f, rates, alpha=0.0, grad=(0.0, 0.0, 0.0), rho0=1.0) -> np.ndarray:
    """MRT collision of one site with an explicit diagonal of 19 rates."""
    g = np.ascontiguousarray(f, dtype=np.float64).copy()
    r = np.ascontiguousarray(rates, dtype=np.float64)
    _load().orc_mrt_collide_site_rates(_ptr(g), float(rho0), _ptr(r), float(alpha), *map(float, grad))
    return g


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


class OracleLattice:
    """Dense FP64 single-fluid lattice (BGK) with the flux inlet / pressure outlet."""

    HIST_FIELDS = ("rho_in", "q_in", "q_out", "mass", "umax")

    def __init__(self, mask: np.ndarray, *, tau: float, q_target: float = 0.0,
                 rho_out: float = 1.0, rho0: float = 1.0, periodic_x: bool = False,
                 periodic_y: bool = False, z_mode: int = Z_FLUX):
        lib = _load()
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.ndim != 3:
            raise ValueError("mask must be (nz, ny, nx)")
        self.shape = mask.shape
        self.mask = mask
        nz, ny, nx = mask.shape
        h = lib.orc_create(nx, ny, nz, _ptr(mask), int(periodic_x), int(periodic_y), int(z_mode),
                           float(tau), float(rho0), float(q_target), float(rho_out))
        if not h:
            raise ValueError("oracle rejected the lattice (dims, tau, rho0 or empty inlet)")
        self._h = h
        self._lib = lib
        self.rho0 = rho0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    @property
    def a_in(self) -> int:
        return int(self._lib.orc_inlet_area(self._h))

    @property
    def a_out(self) -> int:
        return int(self._lib.orc_outlet_area(self._h))

    @property
    def step_count(self) -> int:
        return int(self._lib.orc_step_count(self._h))

    def set_collision(self, on: bool) -> None:
        self._lib.orc_set_collision(self._h, int(bool(on)))

    def set_target_flux(self, q: float) -> None:
        self._lib.orc_set_target_flux(self._h, float(q))

    def set_outlet_density(self, rho: float) -> None:
        self._lib.orc_set_outlet_density(self._h, float(rho))

    def set_mrt(self, on: bool) -> None:
        """MRT collision of Appendix A (single fluid) instead of BGK."""
        self._lib.orc_set_mrt(self._h, int(bool(on)))

    def set_inlet_offset(self, d: float) -> None:
        """Offset added to the inlet density of eq. potential (controller tests)."""
        self._lib.orc_set_inlet_offset(self._h, float(d))

    def plain_inlet_density(self) -> float:
        """The inlet density eq. potential gives for the next step."""
        return float(self._lib.orc_plain_inlet_density(self._h))

    def init_equilibrium(self, rho=1.0, ux=0.0, uy=0.0, uz=0.0) -> None:
        self._lib.orc_init_equilibrium(self._h, float(rho), float(ux), float(uy), float(uz))

    def set_f(self, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != self.shape + (19,):
            raise ValueError("f must be (nz, ny, nx, 19)")
        self._lib.orc_set_f(self._h, _ptr(f))

    def get_f(self) -> np.ndarray:
        out = np.empty(self.shape + (19,), np.float64)
        self._lib.orc_get_f(self._h, _ptr(out))
        return out

    def fields(self):
        """(rho, ux, uy, uz) dense arrays of the stored state."""
        arrs = [np.empty(self.shape, np.float64) for _ in range(4)]
        self._lib.orc_fields(self._h, *[_ptr(a) for a in arrs])
        return tuple(arrs)

    def step(self, n: int = 1, record: bool = True):
        """Advance n steps; returns an (n, 5) history array if record else None."""
        hist = np.empty((n, 5), np.float64) if record else None
        rc = self._lib.orc_step(self._h, int(n), _ptr(hist) if record else None)
        if rc != 0:
            raise RuntimeError("oracle: a population slot was left unset by streaming")
        return hist


class OracleColour:
    """Dense FP64 two-fluid colour-gradient lattice (Appendix A) with the flux
    inlet and pressure outlet. State: f (nz,ny,nx,19), A and B (nz,ny,nx,7)."""

    HIST_FIELDS = ("rho_in", "q_in", "q_out", "mass", "umax", "sum_na", "sum_nb")

    def __init__(self, mask: np.ndarray, *, tau: float, alpha: float, beta: float,
                 phi_solid: float, q_target: float = 0.0, rho_out: float = 1.0,
                 rho0: float = 1.0, periodic_x: bool = False, periodic_y: bool = False,
                 z_mode: int = Z_FLUX):
        lib = _load()
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.shape = mask.shape
        self.mask = mask
        nz, ny, nx = mask.shape
        h = lib.orc_colour_create(nx, ny, nz, _ptr(mask), int(periodic_x), int(periodic_y),
                                  int(z_mode), float(tau), float(rho0), float(q_target),
                                  float(rho_out), float(alpha), float(beta), float(phi_solid))
        if not h:
            raise ValueError("oracle rejected the lattice")
        self._h = h
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_colour_destroy(h)
            self._h = None

    def set_collision(self, on: bool) -> None:
        self._lib.orc_colour_set_collision(self._h, int(bool(on)))

    def init(self, na: np.ndarray, nb: np.ndarray) -> None:
        na = np.ascontiguousarray(na, dtype=np.float64)
        nb = np.ascontiguousarray(nb, dtype=np.float64)
        self._lib.orc_colour_init(self._h, _ptr(na), _ptr(nb))

    def set_state(self, f, A, B) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        A = np.ascontiguousarray(A, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        self._lib.orc_colour_set_state(self._h, _ptr(f), _ptr(A), _ptr(B))

    def get_state(self):
        f = np.empty(self.shape + (19,), np.float64)
        A = np.empty(self.shape + (7,), np.float64)
        B = np.empty(self.shape + (7,), np.float64)
        self._lib.orc_colour_get_state(self._h, _ptr(f), _ptr(A), _ptr(B))
        return f, A, B

    def fields(self):
        """(rho, ux, uy, uz, phi) dense arrays of the stored state."""
        arrs = [np.empty(self.shape, np.float64) for _ in range(5)]
        self._lib.orc_colour_fields(self._h, *[_ptr(a) for a in arrs])
        return tuple(arrs)

    def gradient(self, phi: np.ndarray) -> np.ndarray:
        """Colour gradient (nz, ny, nx, 3) of a dense phase field phi (nz, ny, nx)
        by the stencil the step uses (solid neighbours read phi_solid; zero at
        solid cells)."""
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        if phi.shape != self.shape:
            raise ValueError("phi must be (nz, ny, nx)")
        out = np.empty(self.shape + (3,), np.float64)
        self._lib.orc_colour_gradient(self._h, _ptr(phi), _ptr(out))
        return out

    def step(self, n: int = 1, record: bool = True):
        hist = np.empty((n, 7), np.float64) if record else None
        rc = self._lib.orc_colour_step(self._h, int(n), _ptr(hist) if record else None)
        if rc != 0:
            raise RuntimeError(f"colour oracle step failed ({rc})")
        return hist
