"""ctypes binding of the FP64 oracle in ``lbmref.c`` (test infrastructure only).

Arrays are numpy float64, C-contiguous.  Populations are ``f[a, y, x]`` with
the direction order of Section II (rest, E, N, W, S, NE, NW, SW, SE).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbmref.c")
_LIB = os.path.join(_HERE, "liblbmref.so")

PERIODIC, WALL = 0, 1


def library_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _CParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("omega", ctypes.c_double * 9),
        ("fx", ctypes.c_double),
        ("fy", ctypes.c_double),
        ("force", ctypes.POINTER(ctypes.c_double)),
        ("bc", ctypes.c_int32 * 4),
        ("wall_u", ctypes.c_double * 4),
        ("rho0", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_CParams)
        lib.lbmref_collide.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.lbmref_source.argtypes = [ctypes.c_double] * 4 + [dp]
        lib.lbmref_equilibrium.argtypes = [ctypes.c_double] * 3 + [dp]
        lib.lbmref_kmatrix.argtypes = [dp]
        lib.lbmref_init.argtypes = [pp, dp, dp, dp, dp]
        lib.lbmref_step.argtypes = [pp, dp, dp, ctypes.c_int64]
        lib.lbmref_step_at.argtypes = [pp, dp, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), dp]
        lib.lbmref_macroscopic.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp]
        lib.lbmref_diagnostics.argtypes = [pp, dp, dp]
        lib.lbmref_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params:
    """Problem statement of one lattice (Section II relaxation rates and body
    force; Section III boundary types).  ``bc`` = (x_lo, x_hi, y_lo, y_hi),
    each PERIODIC or WALL; ``wall_u`` = tangential speed of each wall."""

    nx: int
    ny: int
    tau: float = 1.0
    omega3: float = 1.0
    omega6: float = 1.0
    omega7: float = 1.0
    omega8: float = 1.0
    fx: float = 0.0
    fy: float = 0.0
    force: Optional[np.ndarray] = None  # [2, ny, nx] float64
    bc: Sequence[int] = (PERIODIC, PERIODIC, PERIODIC, PERIODIC)
    wall_u: Sequence[float] = (0.0, 0.0, 0.0, 0.0)
    rho0: float = 1.0
    _keep: list = field(default_factory=list, repr=False)

    def omegas(self) -> np.ndarray:
        w = 1.0 / self.tau
        return np.array([0, 0, 0, self.omega3, w, w, self.omega6, self.omega7,
                         self.omega8], dtype=np.float64)

    def c(self) -> _CParams:
        cp = _CParams()
        cp.nx, cp.ny = self.nx, self.ny
        for i, v in enumerate(self.omegas()):
            cp.omega[i] = float(v)
        cp.fx, cp.fy = self.fx, self.fy
        if self.force is not None:
            frc = np.ascontiguousarray(self.force, dtype=np.float64)
            assert frc.shape == (2, self.ny, self.nx)
            self._keep = [frc]
            cp.force = _dp(frc)
        for i in range(4):
            cp.bc[i] = int(self.bc[i])
            cp.wall_u[i] = float(self.wall_u[i])
        cp.rho0 = self.rho0
        return cp


def num_threads() -> int:
    return int(_load().lbmref_num_threads())


def collide(omega: np.ndarray, fx: float, fy: float, fbar: np.ndarray) -> np.ndarray:
    """One node's cascaded collision f-bar -> f~-bar.  ``omega`` has 9 entries
    (indices 3..8 used)."""
    om = np.ascontiguousarray(omega, dtype=np.float64)
    fb = np.ascontiguousarray(fbar, dtype=np.float64)
    out = np.empty(9)
    _load().lbmref_collide(_dp(om), fx, fy, _dp(fb), _dp(out))
    return out


def source(fx: float, fy: float, ux: float, uy: float) -> np.ndarray:
    out = np.empty(9)
    _load().lbmref_source(fx, fy, ux, uy, _dp(out))
    return out


def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.empty(9)
    _load().lbmref_equilibrium(rho, ux, uy, _dp(out))
    return out


def kmatrix() -> np.ndarray:
    out = np.empty(81)
    _load().lbmref_kmatrix(_dp(out))
    return out.reshape(9, 9)


def init_state(p: Params, rho: np.ndarray, ux: np.ndarray, uy: np.ndarray) -> np.ndarray:
    """f-bar(t=0) = f^eq - S/2 from node fields [ny, nx]."""
    r, vx, vy = (np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy))
    f = np.empty((9, p.ny, p.nx))
    cp = p.c()
    _load().lbmref_init(ctypes.byref(cp), _dp(r), _dp(vx), _dp(vy), _dp(f))
    return f


def step(p: Params, f: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance f-bar by ``nsteps`` steps; returns the new array (input kept)."""
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    tmp = np.empty_like(g)
    cp = p.c()
    _load().lbmref_step(ctypes.byref(cp), _dp(g), _dp(tmp), int(nsteps))
    return g


def step_at(p: Params, f: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """f-bar at time n+1 at the listed nodes, from the full state at time n.
    Returns [count, 9]."""
    fb = np.ascontiguousarray(f, dtype=np.float64)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    out = np.empty((len(xs), 9))
    cp = p.c()
    _load().lbmref_step_at(ctypes.byref(cp), _dp(fb), len(xs),
                           xs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           ys.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(out))
    return out


def macroscopic(p: Params, f: np.ndarray) -> dict:
    """rho, ux, uy, sxx, syy, sxy at every node ([ny, nx] each)."""
    fb = np.ascontiguousarray(f, dtype=np.float64)
    outs = {k: np.empty((p.ny, p.nx)) for k in ("rho", "ux", "uy", "sxx", "syy", "sxy")}
    cp = p.c()
    _load().lbmref_macroscopic(ctypes.byref(cp), _dp(fb), *(_dp(outs[k]) for k in
                               ("rho", "ux", "uy", "sxx", "syy", "sxy")))
    return outs


def diagnostics(p: Params, f: np.ndarray) -> np.ndarray:
    """[sum rho, sum rho ux, sum rho uy, 1/2 sum rho |u|^2]."""
    fb = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(4)
    cp = p.c()
    _load().lbmref_diagnostics(ctypes.byref(cp), _dp(fb), _dp(out))
    return out
