"""Oracle: periodic meshes, real FFTs, k-space multipliers and cloud-in-cell (FP64).

TEST INFRASTRUCTURE ONLY. Nothing in the product imports this package.

Paper anchors
-------------
* Sec. 2 and Sec. 2.2: fields live on a grid through cloud-in-cell (CIC) convolution.
* Sec. 5.1, Eq. (priorpdf): the linear modes are Fourier modes with s*(k) = s(-k);
  real and imaginary parts are separate parameters.

Conventions (readings; the paper is silent)
-------------------------------------------
* Grid with n nodes per axis, spacing L/n, node i at position i*L/n.
* Forward DFT unnormalised, X(k) = sum_x x(x) exp(-i k.x); inverse carries 1/n^3.
  Half-spectrum storage [n][n][n/2+1] (numpy rfftn layout).
* Integer wavenumber m = i for i <= n/2, i - n otherwise (last axis 0..n/2);
  k = 2 pi m / L.
* CIC: u = x * (n / L) in FP64, i0 = floor(u) mod n, f = u - floor(u);
  weight (1 - f) on i0 and f on i0 + 1 (mod n), product over axes.
* Cell key of a particle = (i0x * n + i0y) * n + i0z.
"""
import numpy as np


# ------------------------------------------------------------------ k-space

def int_wavenumbers(n):
    """Integer wavenumbers (mx, my, mz) broadcastable to [n][n][n/2+1]."""
    m = np.fft.fftfreq(n, d=1.0 / n)  # 0..n/2-1, -n/2..-1 (exact integers)
    mz = np.arange(n // 2 + 1, dtype=np.float64)
    return m[:, None, None], m[None, :, None], mz[None, None, :]


def wavevectors(n, box):
    mx, my, mz = int_wavenumbers(n)
    c = 2.0 * np.pi / box
    return c * mx, c * my, c * mz


def hermitian_weight(n):
    """Multiplicity of a stored mode in the full spectrum: 1 on mz in {0, n/2}, 2 otherwise."""
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[n // 2] = 1.0
    return np.broadcast_to(w[None, None, :], (n, n, n // 2 + 1))


def gradient_multiplier(n, box, axis):
    """i k_a / k^2: maps the density contrast to the force (and the linear field to the
    Zel'dovich displacement). Zero at k = 0 and on the Nyquist plane of axis a, so that
    the result is the transform of a real field."""
    kv = wavevectors(n, box)
    mv = int_wavenumbers(n)
    k2 = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        mult = 1j * kv[axis] / k2
    mult = np.where(k2 == 0.0, 0.0, mult)
    mult = np.where(np.abs(mv[axis]) == n // 2, 0.0, mult)
    return np.broadcast_to(mult, (n, n, n // 2 + 1))


def hessian_multiplier(n, box, a, b):
    """k_a k_b / k^2: maps the linear field delta to the second derivative phi_{,ab} of the
    potential with laplacian(phi) = delta (phi_hat = -delta_hat / k^2, d_a d_b -> -k_a k_b).
    Zero at k = 0 and on the Nyquist plane of axis a or of axis b (each derivative treated
    as in gradient_multiplier)."""
    kv = wavevectors(n, box)
    mv = int_wavenumbers(n)
    k2 = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        mult = kv[a] * kv[b] / k2
    mult = np.where(k2 == 0.0, 0.0, mult)
    mult = np.where((np.abs(mv[a]) == n // 2) | (np.abs(mv[b]) == n // 2), 0.0, mult)
    return np.broadcast_to(mult, (n, n, n // 2 + 1))


def gaussian_multiplier(n, box, R):
    """exp(-k^2 R^2 / 2): Gaussian smoothing of radius R (Mpc/h); R = 0 is the identity."""
    kv = wavevectors(n, box)
    k2 = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
    return np.exp(-0.5 * k2 * R * R)


def rfft3(field):
    return np.fft.rfftn(field)


def irfft3(spec, n):
    return np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))


def apply_multiplier(field, mult):
    """Real field -> irfft(mult * rfft(field))."""
    n = field.shape[0]
    return irfft3(mult * rfft3(field), n)


def hermitian_project(s):
    """Project stored modes onto the half spectrum of a real field and zero k = 0.

    On the mz = 0 and mz = n/2 planes each stored mode is averaged with the conjugate of
    its partner at (-mx, -my); self-conjugate modes thereby lose their imaginary part.
    (Sec. 5.1: s*(k) = s(-k).)
    """
    n = s.shape[0]
    out = np.array(s, dtype=np.complex128, copy=True)
    neg = (-np.arange(n)) % n
    for iz in (0, n // 2):
        plane = s[:, :, iz]
        partner = plane[neg][:, neg]
        out[:, :, iz] = 0.5 * (plane + np.conj(partner))
    out[0, 0, 0] = 0.0
    return out


# ------------------------------------------------------------------ CIC

def cic_index(x, n, box):
    """Lower CIC corner and fractions. x: (3, P) float64 -> (i0: (3, P) int64, f: (3, P))."""
    u = x * (n / box)
    fl = np.floor(u)
    f = u - fl
    i0 = np.mod(fl.astype(np.int64), n)
    return i0, f


def cell_keys(x, n, box):
    """Cell key of each particle: (i0x * n + i0y) * n + i0z (integer)."""
    i0, _ = cic_index(x, n, box)
    return (i0[0] * n + i0[1]) * n + i0[2]


def sort_order(keys):
    """Particle ids ordered by (cell key, id): the unique stable order."""
    ids = np.arange(keys.size)
    return np.lexsort((ids, keys))


def _corners():
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                yield ox, oy, oz


def cic_paint(x, n, box, values):
    """rho(c) = sum_p values_p * W(x_p - c). values: (P,) or (C, P) -> (n,n,n) or (C,n,n,n)."""
    vals = np.atleast_2d(values)
    i0, f = cic_index(x, n, box)
    out = np.zeros((vals.shape[0], n * n * n))
    for ox, oy, oz in _corners():
        w = ((f[0] if ox else 1.0 - f[0]) * (f[1] if oy else 1.0 - f[1])
             * (f[2] if oz else 1.0 - f[2]))
        idx = (((i0[0] + ox) % n) * n + (i0[1] + oy) % n) * n + (i0[2] + oz) % n
        for c in range(vals.shape[0]):
            out[c] += np.bincount(idx, weights=w * vals[c], minlength=n ** 3)
    out = out.reshape(vals.shape[0], n, n, n)
    return out[0] if np.ndim(values) == 1 else out


def cic_readout(x, n, box, meshes):
    """Interpolate mesh values to particles: v_p = sum_c W(x_p - c) mesh(c).
    meshes: (n,n,n) or (C,n,n,n) -> (P,) or (C,P)."""
    ms = meshes.reshape(-1, n ** 3)
    i0, f = cic_index(x, n, box)
    out = np.zeros((ms.shape[0], x.shape[1]))
    for ox, oy, oz in _corners():
        w = ((f[0] if ox else 1.0 - f[0]) * (f[1] if oy else 1.0 - f[1])
             * (f[2] if oz else 1.0 - f[2]))
        idx = (((i0[0] + ox) % n) * n + (i0[1] + oy) % n) * n + (i0[2] + oz) % n
        out += w[None, :] * ms[:, idx]
    return out[0] if meshes.ndim == 3 else out


def cic_readout_grad(x, n, box, meshes):
    """Position derivative of the CIC readout.

    Returns d[c, a, p] = d/dx_{p,a} sum_cell W(x_p - cell) meshes[c](cell); the weight
    factor along axis a is replaced by its derivative (-n/L on i0, +n/L on i0 + 1).
    """
    ms = meshes.reshape(-1, n ** 3)
    i0, f = cic_index(x, n, box)
    s = n / box
    out = np.zeros((ms.shape[0], 3, x.shape[1]))
    for ox, oy, oz in _corners():
        o = (ox, oy, oz)
        w1 = [f[a] if o[a] else 1.0 - f[a] for a in range(3)]
        dw = [s if o[a] else -s for a in range(3)]
        idx = (((i0[0] + ox) % n) * n + (i0[1] + oy) % n) * n + (i0[2] + oz) % n
        vals = ms[:, idx]
        out[:, 0] += (dw[0] * w1[1] * w1[2])[None] * vals
        out[:, 1] += (w1[0] * dw[1] * w1[2])[None] * vals
        out[:, 2] += (w1[0] * w1[1] * dw[2])[None] * vals
    return out


def lattice_positions(n, box, n_mesh=None):
    """Unperturbed particle positions q on the n^3 lattice, id = (i*n + j)*n + k.

    q_i = i L / n + L / (2 n_mesh): the lattice sits half a force-mesh cell off the mesh
    nodes, so that CIC responds to small displacements with a centred difference (a
    lattice on the nodes gives a one-sided, first-order response)."""
    nm = n if n_mesh is None else n_mesh
    g = np.arange(n) * (box / n) + 0.5 * (box / nm)
    qx, qy, qz = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel(), qz.ravel()])


def wrap(x, box):
    """Periodic wrap of positions into [0, box)."""
    return x - box * np.floor(x / box)
