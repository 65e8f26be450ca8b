"""Python face of liblbm.so: a D2Q9 cascaded-LBM lattice on one GPU.

PyTorch provides the device memory (the two ping-pong lattices, node fields)
and the HIP stream; every step of the method runs in the library's kernels.
The methods below marshal tensors to device pointers and nothing else.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib

_STORAGE_DTYPE = {"fp64": torch.float64, "fp32": torch.float32,
                  "fp16": torch.float16, "bf16": torch.bfloat16}


@dataclass
class Params:
    """Problem statement (Sec. II rates and force, Sec. III boundaries).

    bc: (x_lo, x_hi, y_lo, y_hi), each "periodic" or "wall".
    wall_u: tangential speed of each wall (y-velocity for x walls,
    x-velocity for y walls); a lid is bc[3] = "wall", wall_u[3] = U.
    storage: "fp64", "fp32", "fp16" or "bf16" (the last two store the
    deviations f - w rho0 in 16 bits; arithmetic is FP32).
    rounding: "nearest" (round to nearest even) or "stochastic" (16-bit
    storage only: unbiased stochastic rounding keyed by `seed`).
    """

    nx: int
    ny: int
    tau: float = 1.0
    omega3: float = 1.0
    omega6: float = 1.0
    omega7: float = 1.0
    omega8: float = 1.0
    fx: float = 0.0
    fy: float = 0.0
    bc: Sequence[str] = ("periodic", "periodic", "periodic", "periodic")
    wall_u: Sequence[float] = (0.0, 0.0, 0.0, 0.0)
    rho0: float = 1.0
    storage: str = "fp32"
    rounding: str = "nearest"
    seed: int = 0

    def c(self) -> _lib.LbmParams:
        p = _lib.LbmParams()
        p.nx, p.ny = int(self.nx), int(self.ny)
        p.omega_nu = 1.0 / float(self.tau)
        p.omega3, p.omega6, p.omega7, p.omega8 = (float(v) for v in
                                                  (self.omega3, self.omega6, self.omega7, self.omega8))
        p.fx, p.fy = float(self.fx), float(self.fy)
        for i in range(4):
            b = self.bc[i]
            p.bc[i] = _lib.BC[b] if isinstance(b, str) else int(b)
            p.wall_u[i] = float(self.wall_u[i])
        p.rho0 = float(self.rho0)
        p.storage = _lib.STORAGE[self.storage]
        p.rounding = _lib.ROUNDING[self.rounding]
        p.seed = int(self.seed) & ((1 << 64) - 1)
        return p

    @property
    def real_dtype(self) -> torch.dtype:
        return torch.float64 if self.storage == "fp64" else torch.float32


def lattice_layout(params: Params):
    """(pitch, bytes) of one lattice buffer."""
    pitch, nbytes = ctypes.c_int64(), ctypes.c_int64()
    cp = params.c()
    _lib.check(_lib.lib().lbm_lattice_layout(ctypes.byref(cp), ctypes.byref(pitch), ctypes.byref(nbytes)))
    return pitch.value, nbytes.value


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Lattice:
    """One D2Q9 lattice with its two ping-pong buffers on a GPU.

    State in/out (initial fields, populations, macroscopic fields) is float64
    in every storage mode; the force field, cotangents and gradients use the
    compute real (float64 for "fp64", float32 otherwise)."""

    def __init__(self, params: Params, device="cuda", force: Optional[torch.Tensor] = None,
                 stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("Lattice needs a ROCm GPU (torch.cuda is not available)")
        self.params = params
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.pitch, self.nbytes = lattice_layout(params)
        sdt = _STORAGE_DTYPE[params.storage]
        esz = torch.empty((), dtype=sdt).element_size()
        n = self.nbytes // esz
        self.lat = [torch.zeros(n, dtype=sdt, device=self.device) for _ in range(2)]
        self.real = params.real_dtype
        self.force = None
        if force is not None:
            self.force = self._field(force, (2, params.ny, params.nx))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        cp = params.c()
        _lib.check(_lib.lib().lbm_create(ctypes.byref(cp), _ptr(self.lat[0]), _ptr(self.lat[1]),
                                         _ptr(self.force), ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(ctx)))
        self._ctx = ctx
        self._destroy = _lib.lib().lbm_destroy  # kept: module globals may be gone at exit

    def on_stream(self, stream: torch.cuda.Stream) -> "Lattice":
        """Another handle on this lattice's buffers and force field whose
        library calls launch on `stream` (a context of its own).  Meant for
        the calls that take explicit buffers (step_sequence, step_between,
        the adjoint calls), so that two streams can work on one problem at
        once; its time starts at 0 and it has no state until one is set."""
        v = Lattice.__new__(Lattice)
        v.params, v.device, v.pitch, v.nbytes = self.params, self.device, self.pitch, self.nbytes
        v.lat, v.real, v.force, v.stream = self.lat, self.real, self.force, stream
        ctx = ctypes.c_void_p()
        cp = self.params.c()
        _lib.check(_lib.lib().lbm_create(ctypes.byref(cp), _ptr(v.lat[0]), _ptr(v.lat[1]), _ptr(v.force),
                                         ctypes.c_void_p(stream.cuda_stream), ctypes.byref(ctx)))
        v._ctx = ctx
        v._destroy = _lib.lib().lbm_destroy
        return v

    # ----------------------------------------------------------- plumbing
    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        destroy = getattr(self, "_destroy", None)
        if ctx is not None and ctx.value and destroy is not None:
            destroy(ctx)
            self._ctx = None

    def _check(self, status: int):
        _lib.check(status, self._ctx)

    def _field(self, a, shape, dtype=None) -> torch.Tensor:
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a))
        t = a.to(device=self.device, dtype=self.real if dtype is None else dtype).contiguous()
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def _hold(self, *tensors):
        # Temporaries handed to an asynchronous launch: tell the caching
        # allocator they are in use on the library's stream.
        for t in tensors:
            t.record_stream(self.stream)

    def _after_caller(self):
        # Inputs are produced on the caller's current stream: the library's
        # stream (if another one) waits for them.
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _before_caller(self):
        # Outputs are read on the caller's current stream: it (if another
        # one) waits for the library's work.
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def _lattice_like(self, t: torch.Tensor, what: str):
        if not (t.is_cuda and t.is_contiguous() and t.numel() * t.element_size() >= self.nbytes):
            raise ValueError(f"{what}: need a contiguous device buffer of {self.nbytes} bytes")

    def new_lattice(self) -> torch.Tensor:
        """A zeroed buffer with the layout of one lattice."""
        return torch.zeros_like(self.lat[0])

    def new_cotangent(self) -> torch.Tensor:
        """A zeroed cotangent buffer (compute real, lattice layout)."""
        return torch.zeros(9 * self.params.ny * self.pitch, dtype=self.real, device=self.device)

    @property
    def time(self) -> int:
        return int(_lib.lib().lbm_time(self._ctx))

    @property
    def current(self) -> torch.Tensor:
        ptr = _lib.lib().lbm_current_lattice(self._ctx)
        return self.lat[0] if ptr == self.lat[0].data_ptr() else self.lat[1]

    # --------------------------------------------------------------- state
    def init_equilibrium(self, rho, ux, uy):
        shp = (self.params.ny, self.params.nx)
        r, vx, vy = (self._field(a, shp, torch.float64) for a in (rho, ux, uy))
        self._after_caller()
        self._check(_lib.lib().lbm_init_equilibrium(self._ctx, _ptr(r), _ptr(vx), _ptr(vy)))
        self._hold(r, vx, vy)
        return self

    def set_populations(self, f):
        t = self._field(f, (9, self.params.ny, self.params.nx), torch.float64)
        self._after_caller()
        self._check(_lib.lib().lbm_set_populations(self._ctx, _ptr(t)))
        self._hold(t)
        return self

    def populations(self) -> torch.Tensor:
        out = torch.empty((9, self.params.ny, self.params.nx), dtype=torch.float64, device=self.device)
        self._after_caller()
        self._check(_lib.lib().lbm_get_populations(self._ctx, _ptr(out)))
        self._before_caller()
        return out

    def step(self, n: int = 1):
        self._check(_lib.lib().lbm_step(self._ctx, int(n)))
        return self

    def step_between(self, src: torch.Tensor, dst: torch.Tensor):
        self._lattice_like(src, "src")
        self._lattice_like(dst, "dst")
        self._after_caller()
        self._check(_lib.lib().lbm_step_between(self._ctx, _ptr(src), _ptr(dst)))
        self._before_caller()

    def step_sequence(self, src: torch.Tensor, states: Sequence[torch.Tensor]):
        """states[0] = step(src), states[i] = step(states[i-1]): a segment
        recompute that keeps every state (one native call)."""
        self._lattice_like(src, "src")
        for t in states:
            self._lattice_like(t, "states[i]")
        arr = (ctypes.c_void_p * len(states))(*[t.data_ptr() for t in states])
        self._after_caller()
        self._check(_lib.lib().lbm_step_sequence(self._ctx, _ptr(src), arr, len(states)))
        self._before_caller()

    def snapshot(self, dst: Optional[torch.Tensor] = None) -> torch.Tensor:
        dst = self.new_lattice() if dst is None else dst
        self._lattice_like(dst, "dst")
        self._after_caller()
        self._check(_lib.lib().lbm_snapshot(self._ctx, _ptr(dst)))
        self._before_caller()
        return dst

    def restore(self, src: torch.Tensor, t: int = 0):
        self._lattice_like(src, "src")
        self._after_caller()
        self._check(_lib.lib().lbm_restore(self._ctx, _ptr(src), int(t)))

    def macroscopic(self, strain: bool = True) -> dict:
        shp = (self.params.ny, self.params.nx)
        names = ["rho", "ux", "uy"] + (["sxx", "syy", "sxy"] if strain else [])
        out = {k: torch.empty(shp, dtype=torch.float64, device=self.device) for k in names}
        ptrs = [_ptr(out.get(k)) for k in ("rho", "ux", "uy", "sxx", "syy", "sxy")]
        self._after_caller()
        self._check(_lib.lib().lbm_macroscopic(self._ctx, *ptrs))
        self._before_caller()
        return out

    def diagnostics(self) -> np.ndarray:
        """[sum rho, sum rho ux, sum rho uy, 1/2 sum rho |u|^2] (FP64)."""
        out = (ctypes.c_double * 4)()
        self._check(_lib.lib().lbm_diagnostics(self._ctx, out))
        return np.array(out[:], dtype=np.float64)

    def diagnostics_noalloc(self, out: torch.Tensor) -> torch.Tensor:
        """The same sums into `out` (device float64 [4]), asynchronously on
        the library's stream, with the library's static scratch: no device
        allocation, no synchronisation, no finiteness check."""
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= 4):
            raise ValueError("out: need a contiguous device float64 tensor of 4 elements")
        self._after_caller()
        self._check(_lib.lib().lbm_diagnostics_noalloc(self._ctx, _ptr(out)))
        self._before_caller()
        return out

    # ------------------------------------------------------------- adjoint
    def adjoint_step(self, lat_prev, mu_in, mu_out, grad_force=None):
        self._after_caller()
        self._check(_lib.lib().lbm_adjoint_step(self._ctx, _ptr(lat_prev), _ptr(mu_in), _ptr(mu_out),
                                                _ptr(grad_force)))
        self._before_caller()

    def adjoint_sequence(self, states: Sequence[torch.Tensor], mu_a, mu_b, grad_force=None):
        """Adjoint steps newest-first over states[0..n-1] (mu_a: cotangent of
        the state after the last one).  Returns the buffer, mu_a or mu_b,
        that holds the cotangent of states[0]."""
        arr = (ctypes.c_void_p * len(states))(*[t.data_ptr() for t in states])
        in_b = ctypes.c_int(0)
        self._after_caller()
        self._check(_lib.lib().lbm_adjoint_sequence(self._ctx, arr, len(states), _ptr(mu_a), _ptr(mu_b),
                                                    _ptr(grad_force), ctypes.byref(in_b)))
        self._before_caller()
        return mu_b if in_b.value else mu_a

    def adjoint_macroscopic(self, lat, g_rho, g_ux, g_uy, mu_out, grad_force=None):
        self._after_caller()
        self._check(_lib.lib().lbm_adjoint_macroscopic(self._ctx, _ptr(lat), _ptr(g_rho), _ptr(g_ux),
                                                       _ptr(g_uy), _ptr(mu_out), _ptr(grad_force)))
        self._before_caller()

    def adjoint_init(self, rho, ux, uy, mu0, g_rho=None, g_ux=None, g_uy=None, grad_force=None):
        self._after_caller()
        self._check(_lib.lib().lbm_adjoint_init(self._ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(mu0),
                                                _ptr(g_rho), _ptr(g_ux), _ptr(g_uy), _ptr(grad_force)))
        self._before_caller()
