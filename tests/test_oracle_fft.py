"""Oracle pins: real 3-D DFT conventions, Hermitian projection, k-space multipliers.

The oracle uses numpy's FFT as a step; here it is checked against the O(n^6) definition
of the unnormalised DFT, against Parseval, and against closed forms of single modes.
"""
import numpy as np
import pytest

from oracle import mesh as M


def brute_rdft(x):
    n = x.shape[0]
    idx = np.arange(n)
    out = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    for kx in range(n):
        for ky in range(n):
            for kz in range(n // 2 + 1):
                ph = np.exp(-2j * np.pi * (kx * idx[:, None, None] + ky * idx[None, :, None]
                                           + kz * idx[None, None, :]) / n)
                out[kx, ky, kz] = np.sum(x * ph)
    return out


def brute_irdft(X, n):
    """Inverse from the stored half spectrum, building the full spectrum explicitly."""
    full = np.zeros((n, n, n), dtype=np.complex128)
    for kx in range(n):
        for ky in range(n):
            for kz in range(n):
                if kz <= n // 2:
                    full[kx, ky, kz] = X[kx, ky, kz]
                else:
                    full[kx, ky, kz] = np.conj(X[(-kx) % n, (-ky) % n, n - kz])
    idx = np.arange(n)
    x = np.zeros((n, n, n))
    for i in range(n):
        for j in range(n):
            for k in range(n):
                ph = np.exp(2j * np.pi * (i * idx[:, None, None] + j * idx[None, :, None]
                                          + k * idx[None, None, :]) / n)
                x[i, j, k] = np.real(np.sum(full * ph)) / n ** 3
    return x


@pytest.mark.parametrize("n", [4, 6])
def test_rfft_matches_brute_force_dft(n):
    x = np.random.default_rng(n).standard_normal((n, n, n))
    X = M.rfft3(x)
    np.testing.assert_allclose(X, brute_rdft(x), rtol=0, atol=1e-12 * np.abs(X).max())
    np.testing.assert_allclose(M.irfft3(X, n), brute_irdft(X, n), atol=1e-13)
    np.testing.assert_allclose(M.irfft3(X, n), x, atol=1e-13)


def test_parseval_with_hermitian_weight():
    n = 16
    x = np.random.default_rng(1).standard_normal((n, n, n))
    X = M.rfft3(x)
    lhs = np.sum(x * x)
    rhs = np.sum(M.hermitian_weight(n) * np.abs(X) ** 2) / n ** 3
    assert abs(lhs - rhs) < 1e-12 * lhs


def test_hermitian_projection():
    n = 8
    rng = np.random.default_rng(2)
    s = rng.standard_normal((n, n, n // 2 + 1)) + 1j * rng.standard_normal((n, n, n // 2 + 1))
    p = M.hermitian_project(s)
    # idempotent
    np.testing.assert_allclose(M.hermitian_project(p), p, atol=1e-15)
    # a projected array is the half spectrum of the real field it synthesises
    x = brute_irdft(p, n)
    np.testing.assert_allclose(brute_rdft(x), p, atol=1e-12)
    # self-conjugate modes are real, k = 0 removed
    for i in (0, n // 2):
        for j in (0, n // 2):
            for k in (0, n // 2):
                assert p[i, j, k].imag == 0.0
    assert p[0, 0, 0] == 0.0
    # modes off the mz = 0, n/2 planes are untouched
    np.testing.assert_array_equal(p[:, :, 1:n // 2], s[:, :, 1:n // 2])


def test_gradient_multiplier_single_mode():
    """delta = A cos(k.x) -> F = -A k / k^2 sin(k.x) at the nodes."""
    n, box, A = 16, 100.0, 0.3
    m = np.array([2, -3, 1])
    g = np.arange(n) * box / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    k = 2 * np.pi * m / box
    phase = k[0] * X + k[1] * Y + k[2] * Z
    delta = A * np.cos(phase)
    dk = M.rfft3(delta)
    k2 = np.sum(k * k)
    for a in range(3):
        F = M.irfft3(M.gradient_multiplier(n, box, a) * dk, n)
        np.testing.assert_allclose(F, -A * k[a] / k2 * np.sin(phase), atol=1e-13)


def test_gradient_multiplier_zeroes_nyquist_and_dc():
    n, box = 8, 10.0
    for a in range(3):
        m = M.gradient_multiplier(n, box, a)
        assert m[0, 0, 0] == 0
        sl = [slice(None)] * 3
        sl[a] = n // 2
        assert np.all(m[tuple(sl)] == 0)
        assert np.all(m.real == 0)


def test_gaussian_multiplier_single_mode():
    n, box, R = 16, 64.0, 3.0
    m = np.array([1, 0, 2])
    g = np.arange(n) * box / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    k = 2 * np.pi * m / box
    f = np.cos(k[0] * X + k[1] * Y + k[2] * Z) + 2.0
    out = M.apply_multiplier(f, M.gaussian_multiplier(n, box, R))
    expect = np.exp(-0.5 * np.sum(k * k) * R * R) * (f - 2.0) + 2.0
    np.testing.assert_allclose(out, expect, atol=1e-13)
    np.testing.assert_allclose(M.apply_multiplier(f, M.gaussian_multiplier(n, box, 0.0)), f,
                               atol=1e-13)
