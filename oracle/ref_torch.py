"""Independent float64 PyTorch (CPU) formulation of the cascaded D2Q9 step,
written from the plain definition rather than the paper's explicit kernels.

TEST INFRASTRUCTURE ONLY (gradient reference on tiny grids).

Per node (Sec. II):
  rho = sum f-bar, u = (sum f-bar e + F/2) / rho;
  central moments C_mn = sum_a f-bar_a (e_ax - u_x)^m (e_ay - u_y)^n
  (the discrete central moments defined with the Galilean invariance
  matching principle); each non-conserved central moment relaxes at its own
  rate towards its attractor -- the transformed equilibrium of Sec. II
  (rho, -F_x/2, -F_y/2, rho/3, rho/3, 0, 0, 0, rho/9) before collision and
  rho, +F/2 after (a collision adds the source S, whose central moments are
  (0, F_x, F_y, 0, ...)):
    C*_00 = rho, C*_10 = F_x/2, C*_01 = F_y/2,
    C*_20 + C*_02 = (C_20 + C_02) + w3 (2 rho/3 - (C_20 + C_02)),
    C*_20 - C*_02 = (1 - w4)(C_20 - C_02),  C*_11 = (1 - w5) C_11,
    C*_21 = (1 - w6) C_21,  C*_12 = (1 - w7) C_12,
    C*_22 = C_22 + w8 (rho/9 - C_22);
  f~-bar = the unique D2Q9 vector with these central moments (dense 9x9 solve).
Streaming: pull with periodic wrap, halfway bounce-back and the moving-wall
term 6 rho0 w_a (e_a . U_wall) on links crossing one wall; a link crossing
two walls (through their corner point, at rest) is plain bounce-back
(Sec. III; reading E6).
Initial state: f-bar = (distribution with central moments of the transformed
equilibrium, Sec. II), i.e. f^eq - S/2.

Everything is differentiable by torch autograd with respect to the per-node
force field and the initial velocity.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import torch

EX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
WGT = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
# Moment orders (m, n) in the order 0, x, y, xx, yy, xy, xxy, xyy, xxyy.
ORDERS = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]

_E = torch.tensor([EX, EY], dtype=torch.float64).T  # [9, 2]


def _central_matrix(ux: torch.Tensor, uy: torch.Tensor) -> torch.Tensor:
    """[N, 9, 9]: row (m, n), column a -> (e_ax - ux)^m (e_ay - uy)^n."""
    ex = _E[:, 0][None, :] - ux[:, None]
    ey = _E[:, 1][None, :] - uy[:, None]
    rows = [ex ** m * ey ** n for (m, n) in ORDERS]
    return torch.stack(rows, dim=1)


def _fields(f: torch.Tensor, F: torch.Tensor):
    rho = f.sum(dim=1)
    j = f @ _E + 0.5 * F
    return rho, j[:, 0] / rho, j[:, 1] / rho


def collide(f: torch.Tensor, F: torch.Tensor, omega: Sequence[float]) -> torch.Tensor:
    """f: [N, 9], F: [N, 2]; omega[3..8] used.  Returns f~-bar [N, 9]."""
    rho, ux, uy = _fields(f, F)
    A = _central_matrix(ux, uy)
    C = (A @ f[:, :, None])[:, :, 0]
    w3, w4, w5, w6, w7, w8 = (float(omega[i]) for i in range(3, 9))
    s = C[:, 3] + C[:, 4]
    d = C[:, 3] - C[:, 4]
    s_new = s + w3 * (2.0 / 3.0 * rho - s)
    d_new = (1.0 - w4) * d
    Cn = torch.stack([
        rho, 0.5 * F[:, 0], 0.5 * F[:, 1],
        0.5 * (s_new + d_new), 0.5 * (s_new - d_new),
        (1.0 - w5) * C[:, 5], (1.0 - w6) * C[:, 6], (1.0 - w7) * C[:, 7],
        C[:, 8] + w8 * (rho / 9.0 - C[:, 8]),
    ], dim=1)
    return torch.linalg.solve(A, Cn[:, :, None])[:, :, 0]


def init_state(rho: torch.Tensor, ux: torch.Tensor, uy: torch.Tensor,
               F: torch.Tensor) -> torch.Tensor:
    """Node fields [N] and force [N, 2] -> f-bar(0) [N, 9]."""
    A = _central_matrix(ux, uy)
    z = torch.zeros_like(rho)
    Ceq = torch.stack([rho, -0.5 * F[:, 0], -0.5 * F[:, 1], rho / 3.0, rho / 3.0,
                       z, z, z, rho / 9.0], dim=1)
    return torch.linalg.solve(A, Ceq[:, :, None])[:, :, 0]


def stream_tables(nx: int, ny: int, bc: Sequence[int], wall_u: Sequence[float],
                  rho0: float = 1.0):
    """Gather table for pull streaming.  Populations are flattened as
    index = (y * nx + x) * 9 + a.  Returns (src [9*N] int64, add [9*N])."""
    N = nx * ny
    src = np.empty(9 * N, dtype=np.int64)
    add = np.zeros(9 * N, dtype=np.float64)
    for y in range(ny):
        for x in range(nx):
            for a in range(9):
                sx, sy = x - EX[a], y - EY[a]
                hits = []
                if sx < 0:
                    if bc[0]:
                        hits.append(0)
                    else:
                        sx += nx
                if sx >= nx:
                    if bc[1]:
                        hits.append(1)
                    else:
                        sx -= nx
                if sy < 0:
                    if bc[2]:
                        hits.append(2)
                    else:
                        sy += ny
                if sy >= ny:
                    if bc[3]:
                        hits.append(3)
                    else:
                        sy -= ny
                k = (y * nx + x) * 9 + a
                if hits:
                    src[k] = (y * nx + x) * 9 + OPP[a]
                    if len(hits) == 1:  # two walls: their corner point, at rest
                        h = hits[0]
                        tang = EY[a] if h < 2 else EX[a]
                        add[k] = 6.0 * rho0 * WGT[a] * tang * wall_u[h]
                else:
                    src[k] = (sy * nx + sx) * 9 + a
    return torch.from_numpy(src), torch.from_numpy(add)


def step(f: torch.Tensor, F: torch.Tensor, omega, tables) -> torch.Tensor:
    """One collide-and-stream step on f [N, 9] (node-major)."""
    src, add = tables
    post = collide(f, F, omega).reshape(-1)
    return (post[src] + add).reshape(f.shape)


def velocity(f: torch.Tensor, F: torch.Tensor):
    rho, ux, uy = _fields(f, F)
    return rho, ux, uy


def to_node_major(f_ayx: np.ndarray) -> torch.Tensor:
    """[9, ny, nx] -> [ny*nx, 9]."""
    return torch.from_numpy(np.ascontiguousarray(f_ayx.reshape(9, -1).T))


def to_plane_major(f: torch.Tensor, nx: int, ny: int) -> np.ndarray:
    return f.detach().numpy().T.reshape(9, ny, nx).copy()
