"""Plain-definition helpers the tests use to pin the oracle (numpy, float64).

These are written from the definitions, not from the paper's explicit
formulas, so that agreement between them and the oracle is evidence:
  * central moments C_mn = sum_a f_a (e_ax - u_x)^m (e_ay - u_y)^n;
  * relaxation of each central moment at its own rate (Sec. II, the cascade
    reaches exactly this);
  * inversion by a dense linear solve.
"""
import numpy as np

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
ORDERS = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]


def central_matrix(ux, uy):
    return np.array([(EX - ux) ** m * (EY - uy) ** n for (m, n) in ORDERS])


def fields(f, fx, fy):
    rho = f.sum()
    return rho, (f @ EX + 0.5 * fx) / rho, (f @ EY + 0.5 * fy) / rho


def central_moments(f, ux, uy):
    return central_matrix(ux, uy) @ f


def collide_plain(omega, fx, fy, f):
    """Relax each central moment at its own rate (see module docstring)."""
    rho, ux, uy = fields(f, fx, fy)
    A = central_matrix(ux, uy)
    C = A @ f
    w3, w4, w5, w6, w7, w8 = omega[3:9]
    s, d = C[3] + C[4], C[3] - C[4]
    s2 = s + w3 * (2 * rho / 3 - s)
    d2 = (1 - w4) * d
    Cn = np.array([rho, fx / 2, fy / 2, (s2 + d2) / 2, (s2 - d2) / 2,
                   (1 - w5) * C[5], (1 - w6) * C[6], (1 - w7) * C[7],
                   C[8] + w8 * (rho / 9 - C[8])])
    return np.linalg.solve(A, Cn)


def feq_product(rho, ux, uy):
    """Closed form of the D2Q9 distribution whose central moments are
    (rho, 0, 0, rho/3, rho/3, 0, 0, 0, rho/9): rho phi(e_x, u_x) phi(e_y, u_y),
    phi(0, u) = 2/3 - u^2, phi(+-1, u) = (1/3 + u^2 +- u)/2."""
    def phi(e, u):
        return np.where(e == 0, 2 / 3 - u * u, (1 / 3 + u * u + e * u) / 2)
    return rho * phi(EX, ux) * phi(EY, uy)
