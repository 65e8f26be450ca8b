"""Pins of the oracle's per-node algebra (Sec. II) against the definitions.

No GPU.  Each test checks the oracle against something the paper or the
mathematics fixes independently of the oracle's own formulas.
"""
import os
import zlib

import numpy as np
import pytest

import oracle
from tests import plain

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture
def rng(request):
    # One generator per test, seeded by the test's name, so that a test's
    # draws do not depend on which tests ran before it in the same process.
    return np.random.default_rng(zlib.crc32(request.node.name.encode()))


def _random_case(rng, u_amp=0.1, f_amp=1e-2):
    """A random non-equilibrium population vector, force and rates."""
    f = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4) * (1 + rng.uniform(-0.3, 0.3, 9))
    # add a bulk velocity so u is not small
    f = f + rng.uniform(-u_amp, u_amp) * plain.EX / 9 + rng.uniform(-u_amp, u_amp) * plain.EY / 9
    fx, fy = rng.uniform(-f_amp, f_amp, 2)
    om = np.zeros(9)
    om[3:9] = rng.uniform(0.05, 1.95, 6)
    return f, fx, fy, om


def test_kmatrix_matches_printed():
    """The oracle's K is the matrix printed in Sec. II (golden fixture)."""
    gold = np.loadtxt(os.path.join(GOLDEN, "k_matrix.txt"))
    np.testing.assert_array_equal(oracle.kmatrix(), gold)


def test_kmatrix_columns_are_the_gram_schmidt_basis():
    """Each printed column equals the monomial combination that defines |K_b>
    (Sec. II): K3 = 3|ex^2+ey^2> - 4|1>, K6 = -3|ex^2 ey> + 2|ey>, etc."""
    ex, ey, one = plain.EX, plain.EY, np.ones(9)
    cols = [one, ex, ey, 3 * (ex ** 2 + ey ** 2) - 4 * one, ex ** 2 - ey ** 2, ex * ey,
            -3 * ex ** 2 * ey + 2 * ey, -3 * ex * ey ** 2 + 2 * ex,
            9 * ex ** 2 * ey ** 2 - 6 * (ex ** 2 + ey ** 2) + 4 * one]
    np.testing.assert_array_equal(oracle.kmatrix(), np.stack(cols, axis=1))


def test_k_orthogonality_diagonal():
    """K^T K = D = diag(9, 6, 6, 36, 4, 4, 12, 12, 36) (the orthogonality the
    paper uses to invert K^T S = m^s; reading E1: it is K^T K, not K K^T)."""
    K = oracle.kmatrix()
    np.testing.assert_array_equal(K.T @ K, np.diag([9, 6, 6, 36, 4, 4, 12, 12, 36]).astype(float))


def test_equilibrium_central_moments(rng):
    """f^eq has the Maxwellian central moments (rho, 0, 0, c_s^2 rho, c_s^2 rho,
    0, 0, 0, c_s^4 rho) of Sec. II, and equals the product closed form."""
    for _ in range(20):
        rho = rng.uniform(0.8, 1.2)
        ux, uy = rng.uniform(-0.2, 0.2, 2)
        feq = oracle.equilibrium(rho, ux, uy)
        C = plain.central_moments(feq, ux, uy)
        want = np.array([rho, 0, 0, rho / 3, rho / 3, 0, 0, 0, rho / 9])
        np.testing.assert_allclose(C, want, rtol=0, atol=1e-15)
        np.testing.assert_allclose(feq, plain.feq_product(rho, ux, uy), rtol=0, atol=1e-15)


def test_source_central_moments(rng):
    """The discrete source S_a has central moments (0, F_x, F_y, 0, ..., 0)
    (Sec. II, Galilean invariance matching of sources), for any u."""
    for _ in range(20):
        fx, fy = rng.uniform(-1e-2, 1e-2, 2)
        ux, uy = rng.uniform(-0.2, 0.2, 2)
        S = oracle.source(fx, fy, ux, uy)
        C = plain.central_moments(S, ux, uy)
        np.testing.assert_allclose(C, [0, fx, fy, 0, 0, 0, 0, 0, 0], rtol=0, atol=1e-16)


def test_source_raw_moments_match_binomial():
    """Raw moments of S equal the binomial expansion of its central moments
    about u (Sec. II, binomial formula), e.g. <S|ex^2> = 2 F_x u_x."""
    fx, fy, ux, uy = 3e-3, -2e-3, 0.07, -0.05
    S = oracle.source(fx, fy, ux, uy)
    ex, ey = plain.EX, plain.EY
    np.testing.assert_allclose(S @ (ex ** 2), 2 * fx * ux, atol=1e-17)
    np.testing.assert_allclose(S @ (ex ** 2 * ey), fy * ux ** 2 + 2 * fx * ux * uy, atol=1e-17)
    np.testing.assert_allclose(S @ (ex ** 2 * ey ** 2),
                               2 * fx * ux * uy ** 2 + 2 * fy * uy * ux ** 2, atol=1e-17)


@pytest.mark.parametrize("seed", range(8))
def test_collide_equals_central_moment_relaxation(seed):
    """The paper's explicit cascade (kernels g3..g8 plus S) equals the plain
    definition: every central moment relaxed at its own rate, forcing as
    central moments, inverted by a dense solve.  Random non-equilibrium f,
    random rates in (0, 2), random force."""
    rng = np.random.default_rng(seed)
    for _ in range(50):
        f, fx, fy, om = _random_case(rng)
        got = oracle.collide(om, fx, fy, f)
        want = plain.collide_plain(om, fx, fy, f)
        np.testing.assert_allclose(got, want, rtol=0, atol=2e-15)


def test_collide_fixed_point_of_equilibrium(rng):
    """C(f^eq - S/2) = f^eq + S/2 for any rates: the transformed equilibrium
    is left unchanged by relaxation and gains the full source."""
    for _ in range(20):
        rho = rng.uniform(0.9, 1.1)
        ux, uy = rng.uniform(-0.1, 0.1, 2)
        fx, fy = rng.uniform(-1e-3, 1e-3, 2)
        om = np.zeros(9)
        om[3:9] = rng.uniform(0.1, 1.9, 6)
        feq = plain.feq_product(rho, ux, uy)
        S = oracle.source(fx, fy, ux, uy)
        np.testing.assert_allclose(oracle.collide(om, fx, fy, feq - S / 2), feq + S / 2,
                                   rtol=0, atol=1e-15)


def test_collide_projection_at_unit_rates(rng):
    """With all rates 1 (tau = 1) any input maps to f^eq(rho, u) + S/2."""
    om = np.zeros(9)
    om[3:9] = 1.0
    for _ in range(20):
        f, fx, fy, _ = _random_case(rng)
        rho, ux, uy = plain.fields(f, fx, fy)
        want = plain.feq_product(rho, ux, uy) + oracle.source(fx, fy, ux, uy) / 2
        np.testing.assert_allclose(oracle.collide(om, fx, fy, f), want, rtol=0, atol=2e-15)


def test_collide_conserves_mass_and_adds_force(rng):
    """sum f~ = sum f and sum f~ e = sum f e + F (g0 = g1 = g2 = 0, Sec. II)."""
    for _ in range(50):
        f, fx, fy, om = _random_case(rng)
        out = oracle.collide(om, fx, fy, f)
        assert abs(out.sum() - f.sum()) < 2e-15
        assert abs(out @ plain.EX - (f @ plain.EX + fx)) < 2e-15
        assert abs(out @ plain.EY - (f @ plain.EY + fy)) < 2e-15


def test_collide_unforced_zero_velocity_second_order_relaxation():
    """At u = 0 with F = 0 the shear moment C_11 = <f|ex ey> relaxes by exactly
    (1 - omega_5) and (C_20 - C_02) by (1 - omega_4)."""
    f = plain.feq_product(1.0, 0.0, 0.0)
    f = f.copy()
    f[5] += 1e-3
    f[7] += 1e-3
    f[6] -= 1e-3
    f[8] -= 1e-3  # C_11 = 4e-3, momentum stays 0
    om = np.zeros(9)
    om[3:9] = [1.0, 1.25, 1.25, 1.0, 1.0, 1.0]
    out = oracle.collide(om, 0.0, 0.0, f)
    assert abs((out @ (plain.EX * plain.EY)) - (1 - 1.25) * 4e-3) < 1e-16


def test_x_mirror_equivariance_per_node(rng):
    """Mirroring x (swap E<->W, NE<->NW, SW<->SE, F_x -> -F_x) commutes with
    the collision.  Exact in exact arithmetic; in FP64 the mirrored input is
    summed in another order, so the two sides differ by a few ulps of the
    largest population (a wrong sign on any x-odd term gives ~1e-3)."""
    perm = [0, 3, 2, 1, 4, 6, 5, 8, 7]
    for _ in range(20):
        f, fx, fy, om = _random_case(rng)
        a = oracle.collide(om, fx, fy, f)[perm]
        b = oracle.collide(om, -fx, fy, f[perm])
        np.testing.assert_allclose(a, b, rtol=0, atol=8 * np.finfo(float).eps * np.abs(a).max())
