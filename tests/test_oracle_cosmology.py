"""Oracle pins: growth factors, kick/drift factors and the spectrum normalisation."""
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import cosmology as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_constants():
    out = {}
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, val = line.split()[:2]
                out[name] = float(val)
    return out


def test_paper_omega_m():
    assert C.OMEGA_M_PAPER == _golden_constants()["omega_m"]


@pytest.mark.parametrize("a", [0.1, 0.37, 1.0])
def test_einstein_de_sitter_closed_forms(a):
    # Om = 1: D = a, G_p = a^(3/2)
    assert abs(C.growth_D(a, 1.0) - a) < 1e-12
    assert abs(C.growth_Gp(a, 1.0) - a ** 1.5) < 1e-12


def test_growth_solves_the_linear_growth_ode():
    """Independent route: integrate D'' + (3/a + E'/E) D' = 1.5 Om D / (a^5 E^2) from the
    matter-dominated growing mode (D ~ a) and normalise at a = 1."""
    om = C.OMEGA_M_PAPER
    E = lambda a: np.sqrt(om / a ** 3 + 1 - om)
    dE = lambda a: -1.5 * om / a ** 4 / E(a)

    def rhs(a, y):
        D, dD = y
        return [dD, -(3 / a + dE(a) / E(a)) * dD + 1.5 * om * D / (a ** 5 * E(a) ** 2)]

    a_init = 1e-4
    sol = solve_ivp(rhs, [a_init, 1.0], [a_init, 1.0], rtol=1e-12, atol=1e-16,
                    dense_output=True)
    norm = sol.sol(1.0)[0]
    for a in (0.1, 0.5, 1.0):
        D, dD = sol.sol(a) / norm
        assert abs(C.growth_D(a, om) - D) < 1e-7
        Gp = a ** 3 * E(a) * dD
        assert abs(C.growth_Gp(a, om) - Gp) < 1e-7 * Gp


def test_momentum_growth_identity():
    """dG_p/da = 1.5 Om D / (a^2 E), checked by central differences."""
    om = C.OMEGA_M_PAPER
    for a in (0.12, 0.5, 0.9):
        h = 1e-5
        lhs = (C.growth_Gp(a + h, om) - C.growth_Gp(a - h, om)) / (2 * h)
        rhs = 1.5 * om * C.growth_D(a, om) / (a * a * C.hubble_E(a, om))
        assert abs(lhs - rhs) < 1e-8 * abs(rhs)


@pytest.mark.parametrize("n_steps", [1, 5, 10])
def test_kdk_factors_reproduce_zeldovich_exactly(n_steps):
    """A force that follows linear theory, F(x_i) = D(a_i) Psi, must move every particle
    exactly along x = q + D(a) Psi whatever the step size (Sec. 3: FastPM keeps the
    linear displacement on large scales)."""
    om = C.OMEGA_M_PAPER
    f = C.kdk_factors(0.1, 1.0, n_steps, om)
    psi = np.array([0.7, -1.3, 2.1])
    q = np.array([1.0, 2.0, 3.0])
    x = q + f["D0"] * psi
    p = f["Gp0"] * psi
    for i in range(n_steps):
        p = p + f["kick"][i] * (f["D"][i] * psi)
        x = x + f["drift"][i] * p
    np.testing.assert_allclose(x, q + C.growth_D(1.0, om) * psi, rtol=0, atol=1e-12)


def test_tophat_variance_of_white_noise():
    """P = A: sigma^2(R) = A / (2 pi^2 R^3) int y^2 W^2 dy = 3 A / (4 pi R^3)."""
    A, R = 2.5, 8.0
    s = C.sigma_R(lambda k: A + 0 * k, R, kmin=1e-8, kmax=1e5)
    assert abs(s ** 2 - 3 * A / (4 * np.pi * R ** 3)) < 1e-6 * s ** 2


def test_bbks_normalisation():
    p = C.bbks_power(0.8, 0.2)
    assert abs(C.sigma_R(p, 8.0) - 0.8) < 1e-9
    assert abs(C.bbks_transfer(1e-8) - 1.0) < 1e-6
    assert C.bbks_transfer(0.0) == 1.0
