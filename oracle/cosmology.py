"""Oracle: background cosmology, linear growth and the linear power spectrum (FP64).

TEST INFRASTRUCTURE ONLY. Nothing in the product imports this package.

Paper anchors
-------------
* Sec. 3 (Simulations): flat LambdaCDM with Omega_M = 0.3175; FastPM evolution that
  keeps the linear (Zel'dovich) displacement exact on large scales.
* The paper takes its spectrum from CAMB, which is not available; the synthetic
  stand-in is the BBKS transfer function with Gamma = 0.2, n = 1, sigma8 = 0.8.
* bbks_transfer: parity unpinned. Its coefficients are pinned only by T(0) = 1 and the
  sigma8 normalisation (the publication that defines them is not available here). The
  spectrum only shapes the seeded inputs, which both sides receive identically, so it is
  off the parity path.

Conventions (readings, stated because the paper is silent)
----------------------------------------------------------
Time variable a, Hubble rate in units of H0: E(a) = sqrt(Om a^-3 + 1 - Om).
Growing mode D(a) = C E(a) int_0^a da' / (a' E(a'))^3, normalised to D(1) = 1.
Momentum growth G_p(a) = a^3 E(a) dD/da, which obeys dG_p/da = 1.5 Om D / (a^2 E).
"""
import numpy as np
from scipy import integrate

OMEGA_M_PAPER = 0.3175  # Sec. 3


def hubble_E(a, om):
    return np.sqrt(om * a ** -3.0 + 1.0 - om)


def _dE_da(a, om):
    return -1.5 * om * a ** -4.0 / hubble_E(a, om)


def _growth_integral(a, om):
    f = lambda t: 1.0 / (t * hubble_E(t, om)) ** 3
    val, _ = integrate.quad(f, 0.0, a, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def growth_D(a, om):
    """Linear growing mode, D(1) = 1."""
    norm = hubble_E(1.0, om) * _growth_integral(1.0, om)
    return hubble_E(a, om) * _growth_integral(a, om) / norm


def growth_dD_da(a, om):
    norm = hubble_E(1.0, om) * _growth_integral(1.0, om)
    I = _growth_integral(a, om)
    return (_dE_da(a, om) * I + 1.0 / (a ** 3 * hubble_E(a, om) ** 2)) / norm


def growth_Gp(a, om):
    """G_p = a^3 E dD/da: the momentum of a linear-theory particle per unit displacement."""
    return a ** 3 * hubble_E(a, om) * growth_dD_da(a, om)


def kdk_factors(a0, a1, n_steps, om):
    """Kick/drift factors of an n-step kick-drift-kick scheme uniform in a.

    FastPM-style factors (Sec. 3): each kick integrates dp/da = 1.5 Om F / (a^2 E)
    assuming F grows like D; each drift integrates dx/da = p / (a^3 E) assuming p
    grows like G_p. With these factors a linear force field reproduces the
    Zel'dovich solution exactly for any step size.

    Returns dict with
      D0, Gp0 : growth and momentum factors at a0 (Zel'dovich initial conditions)
      kick[i] : multiplies F(x_i) at force evaluation i (the two half kicks around
                x_i merged; i = 0 has only the half kick a0 -> a_1/2)
      drift[i]: multiplies p_{i+1/2} in x_{i+1} = x_i + drift[i] * p
    """
    a = a0 + (a1 - a0) * np.arange(n_steps + 1) / n_steps
    ah = 0.5 * (a[:-1] + a[1:])
    D = np.array([growth_D(t, om) for t in a])
    Gp = np.array([growth_Gp(t, om) for t in a])
    Gph = np.array([growth_Gp(t, om) for t in ah])
    kick = np.empty(n_steps)
    drift = np.empty(n_steps)
    for i in range(n_steps):
        g_lo = Gp[0] if i == 0 else Gph[i - 1]
        kick[i] = (Gph[i] - g_lo) / D[i]
        drift[i] = (D[i + 1] - D[i]) / Gph[i]
    return {"a": a, "a_half": ah, "D": D, "Gp": Gp, "Gp_half": Gph,
            "D0": D[0], "Gp0": Gp[0], "kick": kick, "drift": drift}


# ---------------------------------------------------------------- spectrum

def bbks_transfer(k, gamma=0.2):
    """BBKS transfer function with shape parameter Gamma, k in h/Mpc (parity unpinned: see
    the module header)."""
    q = np.asarray(k, dtype=np.float64) / gamma
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (np.log1p(2.34 * q) / (2.34 * q)
             * (1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25)
    return np.where(q == 0.0, 1.0, t)


def tophat_window(y):
    """Fourier transform of a unit-volume spherical top hat, W(y) = 3 (sin y - y cos y) / y^3."""
    y = np.asarray(y, dtype=np.float64)
    small = np.abs(y) < 1e-3
    ys = np.where(small, 1.0, y)
    w = 3.0 * (np.sin(ys) - ys * np.cos(ys)) / ys ** 3
    return np.where(small, 1.0 - y * y / 10.0, w)


def sigma_R(power, R, kmin=1e-6, kmax=1e4):
    """rms of the top-hat smoothed field: sigma^2 = (2 pi^2)^-1 int k^2 P(k) W^2(kR) dk."""
    f = lambda lnk: (np.exp(lnk) ** 3 * power(np.exp(lnk)) * tophat_window(np.exp(lnk) * R) ** 2)
    val, _ = integrate.quad(f, np.log(kmin), np.log(kmax), epsabs=0.0, epsrel=1e-11, limit=1000)
    return np.sqrt(val / (2.0 * np.pi ** 2))


def bbks_power(sigma8=0.8, gamma=0.2):
    """Return P(k) = A k T_BBKS(k)^2 normalised to sigma8 (top hat of 8 Mpc/h) at a = 1."""
    shape = lambda k: k * bbks_transfer(k, gamma) ** 2
    s = sigma_R(shape, 8.0)
    A = (sigma8 / s) ** 2
    p = lambda k: A * np.asarray(k, dtype=np.float64) * bbks_transfer(k, gamma) ** 2
    p.amplitude = A
    return p
