"""Particle-mesh force: CIC assignment, Poisson solve with spectral gradient, CIC gather (FP64).

Test infrastructure only (see the package docstring).

Sec. 2.2: the force is computed on a mesh PM_grid times finer per side than the particle
grid, with four FFTs per step -- one to take the density to Fourier space and three to
bring each force component back.  Four FFTs fix a spectral gradient (a real-space
finite-difference gradient would need only two).  The paper does not state the Green's
function, the assignment kernel of the force step, or the mode treatment; the oracle
uses:

  * cloud-in-cell on mesh nodes m*H (H = L / n_g), periodic, unit mass per particle;
    density contrast delta = rho / rho_bar - 1 with rho_bar = N / n_g^3;
  * g = -grad phi with lap phi = delta:  g_k = i k delta_k / k^2 (continuous Green's
    function, spectral gradient, no window deconvolution, no smoothing), k = 0 -> 0 and
    each component zeroed on the Nyquist plane of its own axis;
  * interpolation back to the particles with the same CIC kernel.

The physical acceleration is dp/dt = (3/2) Omega_m g / a (see cola.py).
"""

import numpy as np
from scipy import fft as sfft

from . import lpt


def _cic_corners(pos, n_g, box):
    """For positions (3, N): the 8 corner flat indices (8, N) and weights (8, N)."""
    h = box / n_g
    u = np.mod(np.asarray(pos, dtype=np.float64) / h, n_g)
    m = np.floor(u)
    f = u - m
    m = m.astype(np.int64) % n_g
    idx = []
    wts = []
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                ix = (m[0] + cx) % n_g
                iy = (m[1] + cy) % n_g
                iz = (m[2] + cz) % n_g
                w = ((f[0] if cx else 1.0 - f[0]) * (f[1] if cy else 1.0 - f[1])
                     * (f[2] if cz else 1.0 - f[2]))
                idx.append((ix * n_g + iy) * n_g + iz)
                wts.append(w)
    return np.array(idx), np.array(wts)


def cic_density(pos, n_g, box):
    """Mass per cell (unit particle mass), shape (n_g, n_g, n_g)."""
    idx, wts = _cic_corners(pos, n_g, box)
    rho = np.bincount(idx.ravel(), weights=wts.ravel(), minlength=n_g ** 3)
    return rho.reshape(n_g, n_g, n_g)


def density_contrast(pos, n_g, box):
    """delta = rho / rho_bar - 1 with rho_bar = N / n_g^3."""
    n_part = np.asarray(pos).shape[1]
    rho = cic_density(pos, n_g, box)
    return rho * (n_g ** 3 / n_part) - 1.0


def force_mesh(delta, box):
    """The three components of g = IFFT[i k delta_k / k^2] on the mesh, (3, n, n, n)."""
    n_g = delta.shape[0]
    dk = sfft.rfftn(delta)
    kvec = lpt.wavevectors(n_g, box)
    ik2 = lpt.inverse_k2(kvec[3])
    g = np.empty((3,) + delta.shape)
    for d in range(3):
        g[d] = sfft.irfftn(1j * kvec[d] * ik2 * lpt.nyquist_mask(n_g, d) * dk, s=delta.shape)
    return g


def cic_gather(mesh, pos, box):
    """Interpolate mesh fields (C, n, n, n) to positions (3, N) with CIC; returns (C, N)."""
    n_g = mesh.shape[-1]
    idx, wts = _cic_corners(pos, n_g, box)
    flat = mesh.reshape(mesh.shape[0], -1)
    out = np.zeros((mesh.shape[0], idx.shape[1]))
    for c in range(8):
        out += wts[c] * flat[:, idx[c]]
    return out


def pm_accel(pos, n_g, box):
    """g at the particle positions (3, N): deposit, FFT, Green x gradient, 3 IFFTs, gather."""
    delta = density_contrast(pos, n_g, box)
    g = force_mesh(delta, box)
    return cic_gather(g, pos, box)
