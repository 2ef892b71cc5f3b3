"""Matter power-spectrum estimator (FP64).

Test infrastructure only (see the package docstring).

Sec. 2.5: particles are assigned to a cubic grid with cloud-in-cell, the density is
Fourier transformed, the band power is the average of |delta_k|^2 over the modes of a
k-bin, and the CIC window is deconvolved by a division in Fourier space.  The paper also
names an aliasing correction (Jing 2005) without giving it, and subtracts shot noise only
for haloes; the oracle applies neither to matter.

Redshift-space multipoles (Sec. 6, Eq. 6): the same shells, each mode weighted by
(2 ell + 1) L_ell(mu), mu = m_los / |m| the cosine to the line of sight (plane-parallel along one
axis), L_2 = (3 mu^2 - 1) / 2, L_4 = (35 mu^4 - 30 mu^2 + 3) / 8.

Estimator for an n^3 analysis mesh in a box L:
  delta_k = FFT[rho / rho_bar - 1],
  W(m) = prod_d sinc^2(pi m_d / n)                         (CIC window),
  bin b >= 1 holds the modes with b^2 <= |m|^2 < (b+1)^2  (integer comparison; the
  k = 0 mode is excluded),
  P_b = (L^3 / n^6) sum w |delta_k|^2 / W^2 / sum w,   k_b = sum w |k| / sum w,
where w counts the full k-space from the half spectrum: 2 for 0 < m_z < n/2 and 1 on
the m_z = 0 and m_z = n/2 planes.
"""

import numpy as np
from scipy import fft as sfft

from . import lpt, pm


def mode_weights(n):
    """Full-k-space multiplicity of each half-spectrum mode, shape (1, 1, n/2+1)."""
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    if n % 2 == 0:
        w[-1] = 1.0
    return w[None, None, :]


def cic_window(n):
    """W(m) = prod_d sinc^2(pi m_d / n) on the rfftn grid."""
    mx, my, mz = lpt.mode_integers(n)
    return (np.sinc(mx / n) * np.sinc(my / n) * np.sinc(mz / n)) ** 2


def bin_power(delta_k, n, box, n_bins, deconvolve=True):
    """Bin |delta_k|^2 (half spectrum of an n^3 mesh) into integer-|m| shells.

    Returns (k_mean, pk, n_modes), each of length n_bins; bin 0 is always empty.
    """
    mx, my, mz = lpt.mode_integers(n)
    m2 = mx ** 2 + my ** 2 + mz ** 2
    b = np.floor(np.sqrt(m2.astype(np.float64))).astype(np.int64)
    # exact integer square root: fix the float estimate against b^2 <= m2 < (b+1)^2
    b = np.where(b * b > m2, b - 1, b)
    b = np.where((b + 1) * (b + 1) <= m2, b + 1, b)
    p = np.abs(delta_k) ** 2
    if deconvolve:
        p = p / cic_window(n) ** 2
    w = np.broadcast_to(mode_weights(n), m2.shape)
    kmag = 2.0 * np.pi / box * np.sqrt(m2.astype(np.float64))
    keep = (m2 > 0) & (b < n_bins)
    bb = b[keep]
    ww = w[keep]
    cnt = np.bincount(bb, weights=ww, minlength=n_bins)
    psum = np.bincount(bb, weights=ww * p[keep], minlength=n_bins)
    ksum = np.bincount(bb, weights=ww * kmag[keep], minlength=n_bins)
    with np.errstate(divide="ignore", invalid="ignore"):
        pk = np.where(cnt > 0, psum / cnt * box ** 3 / float(n) ** 6, 0.0)
        km = np.where(cnt > 0, ksum / cnt, 0.0)
    return km, pk, cnt


def power_spectrum(pos, n_mesh, box, n_bins, deconvolve=True):
    """P(k) of particles at positions (3, N) on an n_mesh^3 CIC grid."""
    delta = pm.density_contrast(pos, n_mesh, box)
    dk = sfft.rfftn(delta)
    return bin_power(dk, n_mesh, box, n_bins, deconvolve)


def field_power(delta, box, n_bins):
    """P(k) of a field already on a grid (no assignment window)."""
    n = delta.shape[0]
    dk = sfft.rfftn(delta)
    return bin_power(dk, n, box, n_bins, deconvolve=False)


def legendre(ell, mu):
    """Legendre polynomials L_0, L_2, L_4."""
    mu = np.asarray(mu, dtype=np.float64)
    if ell == 0:
        return np.ones_like(mu)
    if ell == 2:
        return 0.5 * (3.0 * mu ** 2 - 1.0)
    if ell == 4:
        return 0.125 * (35.0 * mu ** 4 - 30.0 * mu ** 2 + 3.0)
    raise ValueError(ell)


def bin_multipoles(delta_k, n, box, n_bins, los=2, deconvolve=True):
    """(k_mean, P_0, P_2, P_4, n_modes) of a half spectrum about axis los, shells of bin_power."""
    mx, my, mz = lpt.mode_integers(n)
    m2 = mx ** 2 + my ** 2 + mz ** 2
    b = np.floor(np.sqrt(m2.astype(np.float64))).astype(np.int64)
    b = np.where(b * b > m2, b - 1, b)
    b = np.where((b + 1) * (b + 1) <= m2, b + 1, b)
    p = np.abs(delta_k) ** 2
    if deconvolve:
        p = p / cic_window(n) ** 2
    ml = (mx, my, mz)[los]
    with np.errstate(divide="ignore", invalid="ignore"):
        mu = np.where(m2 > 0, ml / np.sqrt(m2.astype(np.float64)), 0.0)
    w = np.broadcast_to(mode_weights(n), m2.shape)
    kmag = 2.0 * np.pi / box * np.sqrt(m2.astype(np.float64))
    keep = (m2 > 0) & (b < n_bins)
    bb, ww = b[keep], w[keep]
    cnt = np.bincount(bb, weights=ww, minlength=n_bins)
    ksum = np.bincount(bb, weights=ww * kmag[keep], minlength=n_bins)
    out = []
    for ell in (0, 2, 4):
        s = np.bincount(bb, weights=ww * p[keep] * legendre(ell, mu[keep]), minlength=n_bins)
        with np.errstate(divide="ignore", invalid="ignore"):
            out.append(np.where(cnt > 0, (2 * ell + 1) * s / cnt * box ** 3 / float(n) ** 6, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        km = np.where(cnt > 0, ksum / cnt, 0.0)
    return km, out[0], out[1], out[2], cnt


def multipoles(pos, n_mesh, box, n_bins, los=2, deconvolve=True):
    """Multipoles of particles at positions (3, N) on an n_mesh^3 CIC grid."""
    delta = pm.density_contrast(pos, n_mesh, box)
    return bin_multipoles(sfft.rfftn(delta), n_mesh, box, n_bins, los, deconvolve)
