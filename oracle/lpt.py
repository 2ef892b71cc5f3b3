"""Gaussian initial field and 2LPT displacements (FP64).

Test infrastructure only (see the package docstring).

The paper generates random Gaussian initial conditions with second-order Lagrangian
perturbation theory (Sec. 2.2, citing Crocce, Pueblas & Scoccimarro 2006).  In that
convention the Lagrangian map is

    x(q, a) = q + D1(a) Psi1(q) + D2(a) Psi2(q),
    Psi1 = -grad phi1,   lap phi1 = delta_L        (delta_L: linear field at a = 1)
    Psi2 = +grad phi2,   lap phi2 = sum_{i>j} (phi1_ii phi1_jj - phi1_ij^2)

with D2 ≈ -(3/7) D1^2 < 0.  In Fourier space (k_d = k_f m_d):

    Psi1_k = i k delta_k / k^2,   phi1_ij,k = k_i k_j delta_k / k^2,
    Psi2_k = -i k S_k / k^2,      S = sum_{i>j} (phi1_ii phi1_jj - phi1_ij^2).

Array convention: C order [x][y][z], z fastest; numpy's rfftn halves the z axis.
Mode integers m_d run over [-n/2, n/2).  The k = 0 mode is set to zero.  A multiplier
that is odd in k_d cannot keep a real field real on the Nyquist plane of axis d (where
m_d = -n/2 is its own mirror image), so it is zeroed there; even factors keep it.
"""

import numpy as np
from scipy import fft as sfft

from . import cosmology, noise


def mode_integers(n):
    """Integer wave numbers of an rfftn grid: (mx[:,None,None], my[None,:,None], mz[None,None,:])."""
    m = np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)  # 0..n/2-1, -n/2..-1
    mz = np.arange(n // 2 + 1, dtype=np.int64)
    return m[:, None, None], m[None, :, None], mz[None, None, :]


def wavevectors(n, box):
    """k_x, k_y, k_z (broadcastable) and k^2 on an rfftn grid, k_f = 2 pi / box."""
    kf = 2.0 * np.pi / box
    mx, my, mz = mode_integers(n)
    kx, ky, kz = kf * mx, kf * my, kf * mz
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    return kx, ky, kz, k2


def nyquist_mask(n, axis):
    """1 where the mode is off the Nyquist plane of `axis`, 0 on it (|m_axis| = n/2)."""
    m = mode_integers(n)[axis]
    return (np.abs(m) != n // 2).astype(np.float64)


def inverse_k2(k2):
    """1/k^2 with the k = 0 mode mapped to 0."""
    out = np.zeros_like(k2)
    np.divide(1.0, k2, out=out, where=k2 > 0)
    return out


def gaussian_field_k(n, box, seed, cosmo, amplitude=None):
    """delta_k = FFT[w]_k * sqrt(P(|k|) n^3 / L^3), DC = 0.

    With an unnormalised forward DFT, <|FFT[w]|^2> = n^3, so <|delta_k|^2> = n^6 P / L^3
    and the estimator (L^3 / n^6) |delta_k|^2 is unbiased for P.
    """
    w = noise.white_noise(n, seed)
    wk = sfft.rfftn(w)
    _, _, _, k2 = wavevectors(n, box)
    pk = cosmology.linear_power(np.sqrt(k2), cosmo, amplitude)
    dk = wk * np.sqrt(pk * n ** 3 / box ** 3)
    dk[0, 0, 0] = 0.0
    return dk


def first_order(delta_k, n, box):
    """Psi1 (3, n, n, n) from delta_k: Psi1_d = IFFT[i k_d delta_k / k^2]."""
    kvec = wavevectors(n, box)
    ik2 = inverse_k2(kvec[3])
    psi = np.empty((3, n, n, n))
    for d in range(3):
        psi[d] = sfft.irfftn(1j * kvec[d] * ik2 * nyquist_mask(n, d) * delta_k, s=(n, n, n))
    return psi


def second_order_source(delta_k, n, box):
    """S = sum_{i>j} (phi_ii phi_jj - phi_ij^2), phi_ij = IFFT[k_i k_j delta_k / k^2]."""
    kvec = wavevectors(n, box)
    ik2 = inverse_k2(kvec[3])

    def phi(i, j):
        mult = kvec[i] * kvec[j] * ik2
        if i != j:
            mult = mult * nyquist_mask(n, i) * nyquist_mask(n, j)
        return sfft.irfftn(mult * delta_k, s=(n, n, n))

    pxx, pyy, pzz = phi(0, 0), phi(1, 1), phi(2, 2)
    pxy, pxz, pyz = phi(0, 1), phi(0, 2), phi(1, 2)
    return pxx * pyy + pxx * pzz + pyy * pzz - pxy ** 2 - pxz ** 2 - pyz ** 2


def second_order(delta_k, n, box):
    """Psi2 (3, n, n, n): Psi2_d = IFFT[-i k_d S_k / k^2]."""
    s = second_order_source(delta_k, n, box)
    sk = sfft.rfftn(s)
    kvec = wavevectors(n, box)
    ik2 = inverse_k2(kvec[3])
    psi = np.empty((3, n, n, n))
    for d in range(3):
        psi[d] = sfft.irfftn(-1j * kvec[d] * ik2 * nyquist_mask(n, d) * sk, s=(n, n, n))
    return psi


def lagrangian_grid(n, box):
    """q = (i, j, l) * box / n, shape (3, n, n, n): particles start at cell corners."""
    g = np.arange(n, dtype=np.float64) * (box / n)
    qx, qy, qz = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([qx, qy, qz])


def initial_conditions(n, box, seed, cosmo, a_init, amplitude=None):
    """2LPT initial state at a_init.

    Returns dict with psi1, psi2 (3, n, n, n) at D1 = 1 and the displacement
    disp = D1(a_init) Psi1 + D2(a_init) Psi2 from the Lagrangian position.
    """
    dk = gaussian_field_k(n, box, seed, cosmo, amplitude)
    psi1 = first_order(dk, n, box)
    psi2 = second_order(dk, n, box)
    d1, d2 = cosmology.growth_factors([a_init], cosmo.omega_m)[:2, 0]
    disp = d1 * psi1 + d2 * psi2
    return {"delta_k": dk, "psi1": psi1, "psi2": psi2, "disp": disp, "d1": d1, "d2": d2}
