"""Matter power-spectrum estimator (FP64).

Test infrastructure only (see the package docstring).

Sec. 2.5: particles are assigned to a cubic grid with cloud-in-cell, the density is
Fourier transformed, the band power is the average of |delta_k|^2 over the modes of a
k-bin, and the CIC window is deconvolved by a division in Fourier space.  The paper also
corrects for aliasing as in Jing (2005) without giving the method: bin_power is the plain
deconvolved estimator, bin_power_corrected the estimator with that correction (the aliasing
sum of a local power law, the slope iterated from the estimate itself; see its docstring).
Shot noise is not subtracted for matter (the paper subtracts it only for haloes).

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


# --------------------------------------------------------------------------- aliasing correction

def aliasing_sum(n, n_eff, images=2):
    """Per mode of the rfftn grid of an n^3 mesh, the CIC aliasing sum of Jing (2005) for a local
    power law P(k) ~ k^n_eff:

      C(m) = sum_{j in Z^3, |j_d| <= images} W^2(u_j) (|u_j| / |m|)^n_eff,   u_j = |m| + j n
      W(u) = prod_d sinc^2(pi u_d / n)  (CIC),  |m| = (|m_x|, |m_y|, |m_z|);

    the measured <|delta_m|^2> is C(m) P(|m|) when the spectrum is a power law near |m| (the j = 0
    term alone is the window deconvolution).  The images are taken about the absolute mode
    integers so that C has the symmetry of the mesh also on the Nyquist planes, where the truncated
    image set of -n/2 and of +n/2 would otherwise differ.  n_eff: scalar or an array broadcast over
    the modes.  The dropped images fall off as (j_d)^-4 (at n_eff = 0 the untruncated sum is the
    closed form prod_d [1 - (2/3) sin^2(pi m_d / n)]).  k = 0 gets C = 1."""
    m = [np.abs(np.asarray(v, dtype=np.float64)) for v in lpt.mode_integers(n)]
    m2 = m[0] ** 2 + m[1] ** 2 + m[2] ** 2
    shape = np.broadcast(m[0], m[1], m[2]).shape
    n_eff = np.broadcast_to(np.asarray(n_eff, dtype=np.float64), shape)
    s2 = [np.sin(np.pi * v / n) ** 2 for v in m]  # sin^2(pi (m_d + j n) / n) does not depend on j
    safe_m2 = np.where(m2 > 0, m2, 1.0)
    total = np.zeros(shape)
    with np.errstate(divide="ignore"):  # k = 0 (a2 = 0 at j = 0) is replaced below
        _image_sum(total, m, s2, safe_m2, n, n_eff, images)
    return np.where(m2 > 0, total, 1.0)


def _image_sum(total, m, s2, safe_m2, n, n_eff, images):
    """Adds the images |j_d| <= images of aliasing_sum into total."""
    shape = total.shape
    for jx in range(-images, images + 1):
        for jy in range(-images, images + 1):
            for jz in range(-images, images + 1):
                w2 = np.ones(shape)
                a2 = np.zeros(shape)
                for d, jd in enumerate((jx, jy, jz)):
                    u = m[d] + jd * n  # image mode integer
                    x = np.pi * u / n
                    w2 = w2 * np.where(u == 0, 1.0, (s2[d] / np.where(u == 0, 1.0, x * x)) ** 2)
                    a2 = a2 + u * u
                total += w2 * (a2 / safe_m2) ** (0.5 * n_eff)


def local_slopes(k, pk, n_modes, width=1.35):
    """d ln P / d ln k in each bin: the least-squares slope of ln P against ln k over the non-empty
    bins with k_b / width <= k <= k_b width, each weighted by its mode count (a window in log k
    rather than the two neighbours keeps the slope of a noisy estimate, and with it the iteration,
    stable near the mesh corners).  Clamped to [-4, 4]; 0 where the window holds fewer than two
    bins or the bin is empty."""
    ok = (k > 0) & (pk > 0)
    lk = np.log(np.where(ok, k, 1.0))
    lp = np.log(np.where(ok, pk, 1.0))
    out = np.zeros(len(k))
    for b in np.nonzero(ok)[0]:
        sel = ok & (k >= k[b] / width) & (k <= k[b] * width)
        if sel.sum() < 2:
            continue
        w, x, y = n_modes[sel], lk[sel], lp[sel]
        xm, ym = np.average(x, weights=w), np.average(y, weights=w)
        out[b] = np.sum(w * (x - xm) * (y - ym)) / np.sum(w * (x - xm) ** 2)
    return np.clip(out, -4.0, 4.0)


def bin_power_corrected(delta_k, n, box, n_bins, iterations=4, images=2):
    """Sec. 2.5 with the aliasing correction of Jing (2005): start from the window-deconvolved
    estimate (bin_power), then repeat `iterations` times: take the local slope n_eff of the current
    estimate in each bin (local_slopes), divide every mode's |delta_m|^2 by its aliasing sum C(m)
    for the slope of its bin (instead of by W^2 alone) and bin again.  Shot noise is part of the
    measured power and is corrected with it (a flat spectrum has n_eff = 0, whose aliasing sum is
    the closed form of the CIC shot noise).  Returns (k_mean, pk, n_modes)."""
    km, pk, cnt = bin_power(delta_k, n, box, n_bins)
    mx, my, mz = lpt.mode_integers(n)
    m2 = mx ** 2 + my ** 2 + mz ** 2
    b = np.floor(np.sqrt(m2.astype(np.float64))).astype(np.int64)
    b = np.where(b * b > m2, b - 1, b)
    b = np.where((b + 1) * (b + 1) <= m2, b + 1, b)
    keep = (m2 > 0) & (b < n_bins)
    bb = np.where(keep, b, 0)
    p = np.abs(delta_k) ** 2
    w = np.broadcast_to(mode_weights(n), m2.shape)
    for _ in range(iterations):
        slope = local_slopes(km, pk, cnt)
        c = aliasing_sum(n, slope[bb], images)
        psum = np.bincount(bb[keep], weights=(w * p / c)[keep], minlength=n_bins)
        with np.errstate(divide="ignore", invalid="ignore"):
            pk = np.where(cnt > 0, psum / cnt * box ** 3 / float(n) ** 6, 0.0)
    return km, pk, cnt


def power_spectrum_corrected(pos, n_mesh, box, n_bins, iterations=4, images=2):
    """P(k) of particles at positions (3, N) on an n_mesh^3 CIC grid with the aliasing correction."""
    delta = pm.density_contrast(pos, n_mesh, box)
    return bin_power_corrected(sfft.rfftn(delta), n_mesh, box, n_bins, iterations, images)
