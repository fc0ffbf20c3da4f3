"""Oracle: binned two-point statistics (Sec. 4.3, two point functions: the
cross-correlation coefficient, the stochasticity and the transfer function per k bin),
used to score a reconstruction against the true linear field, in FP64 with plain numpy.

TEST INFRASTRUCTURE ONLY. Nothing in the product imports this package.

For two fields stored as rfft half spectra a, b on an n^3 mesh of side L, and shells
k in [i dk, (i + 1) dk) with dk = 2 pi / L (the fundamental), i = 0 .. nbins - 1:
  count_i = number of full-spectrum modes in the shell (the k = 0 mode excluded),
  P_aa(i) = L^3 / n^6 * mean |a|^2,  P_bb(i) = L^3 / n^6 * mean |b|^2,
  P_ab(i) = L^3 / n^6 * mean Re(a conj(b)),
the means taken over the full spectrum (each stored mode off the kz = 0 and n/2 planes
stands for itself and its conjugate partner, weight 2). Then
  r_c = P_ab / sqrt(P_aa P_bb),  s = P_aa (1 - r_c^2),  TF = sqrt(P_bb / P_aa)
with a the reference (true) field and b the model (reconstructed) field.
"""
import numpy as np

from . import mesh as M


def power_bins(a, b, box, nbins):
    """-> (count, P_aa, P_bb, P_ab), each [nbins] (FP64)."""
    n = a.shape[0]
    mx, my, mz = M.int_wavenumbers(n)
    m2 = np.broadcast_to(mx ** 2 + my ** 2 + mz ** 2, a.shape)  # exact integers
    w = np.broadcast_to(M.hermitian_weight(n), a.shape)
    # shell of |k| in units of dk = 2 pi / L: floor(sqrt(m^2)), exact for perfect squares
    idx = np.floor(np.sqrt(m2)).astype(np.int64)
    use = (m2 > 0) & (idx < nbins)
    cnt = np.zeros(nbins)
    paa = np.zeros(nbins)
    pbb = np.zeros(nbins)
    pab = np.zeros(nbins)
    ii = idx[use]
    ww = w[use]
    av, bv = a[use], b[use]
    np.add.at(cnt, ii, ww)
    np.add.at(paa, ii, ww * np.abs(av) ** 2)
    np.add.at(pbb, ii, ww * np.abs(bv) ** 2)
    np.add.at(pab, ii, ww * (av.real * bv.real + av.imag * bv.imag))
    norm = box ** 3 / float(n) ** 6
    with np.errstate(invalid="ignore", divide="ignore"):
        scale = np.where(cnt > 0, norm / np.where(cnt > 0, cnt, 1.0), 0.0)
    return cnt, paa * scale, pbb * scale, pab * scale


def metrics(paa, pbb, pab):
    """-> (r_c, stochasticity, TF) per bin (0 where a spectrum is empty)."""
    with np.errstate(invalid="ignore", divide="ignore"):
        ok = paa * pbb > 0
        rc = np.where(ok, pab / np.sqrt(np.where(ok, paa * pbb, 1.0)), 0.0)
        tf = np.where(paa > 0, np.sqrt(np.where(paa > 0, pbb / np.where(paa > 0, paa, 1.0), 0.0)), 0.0)
    return rc, paa * (1.0 - rc ** 2), tf
