"""Python access to the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg use this module.  The GPU library and its
binding never import it.

The oracle is plain C compiled with gcc into ``liboracle.so`` next to this
file; :func:`build` compiles it, and :func:`lib` compiles it on first use
when no build exists yet.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

OUTFLOW = 0
PERIODIC = 1


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (plain -O2, one thread)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, _SRC, "-lm"], cwd=_HERE)
        os.replace(tmp, _SO)
    return _SO


class _Cfg(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("q_phi", ctypes.c_int), ("q_chi", ctypes.c_int), ("K", ctypes.c_int),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int)]


@dataclass
class Config:
    d: int
    nx: int
    ny: int = 1
    lx: float = 1.0
    ly: float = 1.0
    q_phi: int = 5
    q_chi: int = 3
    K: int = 2
    tau: float = 1e-5
    dt: float = 1e-4
    bc_x: int = OUTFLOW
    bc_y: int = OUTFLOW

    def _c(self) -> _Cfg:
        return _Cfg(self.d, self.nx, self.ny if self.d == 2 else 1, self.lx, self.ly,
                    self.q_phi, self.q_chi, self.K, self.tau, self.dt, self.bc_x, self.bc_y)

    @property
    def cells(self) -> int:
        return self.nx * (self.ny if self.d == 2 else 1)

    @property
    def planes(self) -> int:
        return self.q_phi ** self.d + self.q_chi ** self.d

    @property
    def shape(self):
        """Shape of a state array: (planes, ny, nx) or (planes, nx)."""
        if self.d == 2:
            return (self.planes, self.ny, self.nx)
        return (self.planes, self.nx)

    @property
    def field_shape(self):
        return (self.ny, self.nx) if self.d == 2 else (self.nx,)


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        cp = ctypes.POINTER(_Cfg)
        L.oracle_num_planes.argtypes = [cp]
        L.oracle_gauss_hermite.argtypes = [ctypes.c_int, _dp, _dp]
        L.oracle_g.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_velocities.argtypes = [cp, _dp, _dp]
        L.oracle_equilibrium.argtypes = [cp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_moments.argtypes = [cp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_mp9_face.argtypes = [_dp]
        L.oracle_mp9_face.restype = ctypes.c_double
        L.oracle_advect.argtypes = [cp, _dp, _dp]
        L.oracle_step.argtypes = [cp, _dp, ctypes.c_int, _dp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def gauss_hermite(Q: int):
    p = np.zeros(Q)
    w = np.zeros(Q)
    if lib().oracle_gauss_hermite(Q, _ptr(p), _ptr(w)) != 0:
        raise ValueError(f"quadrature order {Q} not supported")
    return p, w


def g_factor(Q: int, u: float, T: float) -> np.ndarray:
    p, w = gauss_hermite(Q)
    g = np.zeros(Q)
    lib().oracle_g(Q, _ptr(p), _ptr(w), float(u), float(T), _ptr(g))
    return g


def velocities(cfg: Config):
    px = np.zeros(cfg.planes)
    py = np.zeros(cfg.planes)
    c = cfg._c()
    lib().oracle_velocities(ctypes.byref(c), _ptr(px), _ptr(py))
    return px, py


def equilibrium(cfg: Config, n, ux, uy, T) -> np.ndarray:
    n, ux, T = _f64(n), _f64(ux), _f64(T)
    uy = _f64(uy) if uy is not None else np.zeros_like(n)
    F = np.zeros(cfg.shape)
    c = cfg._c()
    lib().oracle_equilibrium(ctypes.byref(c), _ptr(n), _ptr(ux), _ptr(uy), _ptr(T), _ptr(F))
    return F


def moments(cfg: Config, F):
    F = _f64(F)
    assert F.shape == cfg.shape
    n = np.zeros(cfg.field_shape)
    ux = np.zeros(cfg.field_shape)
    uy = np.zeros(cfg.field_shape)
    T = np.zeros(cfg.field_shape)
    c = cfg._c()
    lib().oracle_moments(ctypes.byref(c), _ptr(F), _ptr(n), _ptr(ux), _ptr(uy), _ptr(T))
    return n, ux, uy, T


def mp9_face(f9) -> float:
    f9 = _f64(f9)
    assert f9.shape == (9,)
    return lib().oracle_mp9_face(_ptr(f9))


def advect(cfg: Config, F) -> np.ndarray:
    F = _f64(F)
    assert F.shape == cfg.shape
    VF = np.zeros(cfg.shape)
    c = cfg._c()
    lib().oracle_advect(ctypes.byref(c), _ptr(F), _ptr(VF))
    return VF


def step(cfg: Config, F, nsteps: int = 1, with_stages: bool = False):
    """Return F after ``nsteps`` IMEX steps (and the last step's stages)."""
    F = np.array(F, dtype=np.float64, order="C", copy=True)
    assert F.shape == cfg.shape
    stages = np.zeros((4,) + cfg.shape) if with_stages else None
    c = cfg._c()
    rc = lib().oracle_step(ctypes.byref(c), _ptr(F), int(nsteps),
                           _ptr(stages) if with_stages else None)
    if rc != 0:
        raise ValueError("oracle_step rejected the configuration")
    return (F, stages) if with_stages else F
