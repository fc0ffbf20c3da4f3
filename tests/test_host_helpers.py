"""The product's host-side input helpers agree with the oracle's independent versions."""
import numpy as np

import synth
from oracle import cosmology as OC
from oracle import model as OM
from paper_1805_02247_amd import cosmo


def test_spectrum_normalisation_agrees():
    P1 = cosmo.linear_power(0.8, 0.2)
    P2 = OC.bbks_power(0.8, 0.2)
    k = np.logspace(-3, 1, 50)
    np.testing.assert_allclose(P1(k), P2(k), rtol=1e-6)


def test_prior_table_and_modes_agree():
    n, box = 16, 100.0
    P = OC.bbks_power()
    inv1 = cosmo.prior_inv_variance(n, box, P)
    inv2 = OM.prior_inv_variance(n, box, P)
    np.testing.assert_allclose(inv1, inv2, rtol=1e-6)
    w = synth.white_noise(3, n)
    s1 = cosmo.modes_from_white_noise(w, box, P)
    s2 = OM.linear_modes(w, box, P)
    np.testing.assert_allclose(s1, s2, rtol=1e-5, atol=1e-6 * np.abs(s2).max())
