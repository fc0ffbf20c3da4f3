"""Host-side set-up helpers: linear power spectrum, prior table and Gaussian linear modes.

These run once per configuration on the host (numpy, FP64) and only prepare inputs of the
device path: the prior inverse variance 1/S(k) and the initial modes s(k). The forward
model and its gradient never run here.

Spectrum: P(k) = A k T(k)^2 with the BBKS transfer function (shape Gamma), normalised to
sigma8 with a spherical top hat of 8 Mpc/h (the paper uses CAMB with the cosmology of its
Sec. 3; BBKS is the synthetic stand-in).
"""
import numpy as np


def _transfer(k, gamma):
    q = np.maximum(np.asarray(k, dtype=np.float64), 1e-300) / gamma
    return (np.log1p(2.34 * q) / (2.34 * q)
            * (1 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25)


def _tophat(y):
    y = np.asarray(y, dtype=np.float64)
    ys = np.where(y < 1e-3, 1.0, y)
    return np.where(y < 1e-3, 1 - y * y / 10, 3 * (np.sin(ys) - ys * np.cos(ys)) / ys ** 3)


def linear_power(sigma8=0.8, gamma=0.2):
    """Returns P(k) (k in h/Mpc, P in (Mpc/h)^3) normalised to sigma8 at a = 1."""
    lnk = np.linspace(np.log(1e-6), np.log(1e4), 400001)
    k = np.exp(lnk)
    integrand = k ** 3 * k * _transfer(k, gamma) ** 2 * _tophat(8.0 * k) ** 2
    s2 = np.sum(0.5 * (integrand[1:] + integrand[:-1]) * np.diff(lnk)) / (2 * np.pi ** 2)
    A = sigma8 ** 2 / s2

    def P(kk):
        kk = np.asarray(kk, dtype=np.float64)
        return A * kk * _transfer(kk, gamma) ** 2

    P.amplitude = A
    return P


def _kmag(n, box):
    m = np.fft.fftfreq(n, d=1.0 / n)
    mz = np.arange(n // 2 + 1)
    c = 2 * np.pi / box
    return c * np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 + mz[None, None, :] ** 2)


def prior_inv_variance(n, box, power):
    """float32 [n][n][n/2+1]: 1/S(k), S = n^6 P(k) / box^3 (unnormalised DFT); 0 at k = 0."""
    k = _kmag(n, box)
    with np.errstate(divide="ignore"):
        inv = box ** 3 / (n ** 6 * power(np.where(k == 0, 1.0, k)))
    inv[0, 0, 0] = 0.0
    return inv.astype(np.float32)


def modes_from_white_noise(white, box, power):
    """complex64 [n][n][n/2+1]: s = rfft(w) sqrt(n^3 P(k) / box^3), s(0) = 0."""
    n = white.shape[0]
    k = _kmag(n, box)
    s = np.fft.rfftn(white) * np.sqrt(n ** 3 * power(np.where(k == 0, 1.0, k)) / box ** 3)
    s[0, 0, 0] = 0
    return s.astype(np.complex64)
