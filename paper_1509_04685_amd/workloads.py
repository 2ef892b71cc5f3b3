"""Synthetic workloads: problem sizes, cosmology, seeds and seeded random inputs.

This module holds no arithmetic of the method; it only names the configurations and draws
seeded random numbers, so that the library, the float64 oracle (in the tests) and the
benchmark all see identical inputs.

Every workload is a Gaussian random field with a BBKS spectrum in the MICE-GC cosmology of
Sec. 2.1 (Omega_m 0.25, Omega_b 0.044, h 0.7, n_s 0.95, sigma_8 0.8); these synthetic fields stand
in for the paper's CAMB spectrum and for MICE-GC itself, which are not available.  Sizes follow
the paper's optimum (Sec. 4.5: 40 nodes linear in a from z_i = 19, PM_grid = 3) scaled to one GPU.
"""

import numpy as np

COSMOLOGY = dict(omega_m=0.25, omega_b=0.044, h=0.7, n_s=0.95, sigma_8=0.8)

# name: (box [h^-1 Mpc], N_p, PM_grid, z_init, n_steps, seeds)
CONFIGS = {
    # small case: 32^3 particles, 96^3 mesh, 10 nodes from z = 19
    "plain_32_96": dict(box=256.0, n_part=32, pm_factor=3, z_init=19.0, n_steps=10, seeds=(1, 2, 3)),
    # the headline case: 256^3 particles, 768^3 mesh, 40 nodes from z = 19, P(k) at z = 1, 0.5, 0
    "plain_256_768": dict(box=768.0, n_part=256, pm_factor=3, z_init=19.0, n_steps=40, seeds=(1,),
                          a_out=(0.5, 1.0 / 1.5, 1.0)),
    # ensemble shape classes: 24 x (96^3 / 288^3, L 300) and 24 x (128^3 / 384^3, L 400)
    "ens_96_288": dict(box=300.0, n_part=96, pm_factor=3, z_init=19.0, n_steps=40,
                       seeds=tuple(range(1001, 1025))),
    "ens_128_384": dict(box=400.0, n_part=128, pm_factor=3, z_init=19.0, n_steps=40,
                        seeds=tuple(range(2001, 2025))),
    # coarse 1x mesh with the learned correction
    "learned_256_256": dict(box=768.0, n_part=256, pm_factor=1, z_init=19.0, n_steps=40, seeds=(1,)),
    # large: 512^3 particles, 1536^3 mesh
    "plain_512_1536": dict(box=1536.0, n_part=512, pm_factor=3, z_init=19.0, n_steps=40, seeds=(1,),
                           a_out=(1.0,)),
    # the learned form beside it: 512^3 particles on the 512^3 mesh (same 3 h^-1 Mpc cells)
    "learned_512_512": dict(box=1536.0, n_part=512, pm_factor=1, z_init=19.0, n_steps=40, seeds=(1,)),
}


def uniform_positions(n, box, seed):
    """(3, n) float64 positions uniform in [0, box)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, box, size=(3, n))


def clustered_positions(n, box, seed, n_clumps=8, frac=0.5, width=2.0):
    """(3, n) positions: a uniform part plus Gaussian clumps (a crude stand-in for haloes)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(3, n))
    k = int(frac * n)
    centres = rng.uniform(0.0, box, size=(3, n_clumps))
    which = rng.integers(0, n_clumps, size=k)
    pos[:, :k] = centres[:, which] + rng.normal(0.0, width, size=(3, k))
    return np.mod(pos, box)


def random_field(n, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n, n)).astype(dtype)


def random_displacements(n_part, scale, seed):
    """(3, n_part^3) displacements, Gaussian with the given rms per axis."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=(3, n_part ** 3))


def halo_positions(n, box, seed, n_halo, halo_frac=0.5, halo_radius=1.0, slope=-1.9, min_members=2):
    """(3, n) float32 positions in [0, box) with a halo population: a fraction halo_frac of the
    particles in n_halo spherical clumps whose member counts follow a power law dN/dm ~ m^slope
    (as a halo mass function does below its knee) and whose Plummer-like profiles have scale
    radius halo_radius * (m / mean m)^(1/3); the rest uniform.  Particle order is shuffled so that
    members of one clump are not neighbours in index."""
    rng = np.random.default_rng(seed)
    n_in = int(halo_frac * n)
    if n_halo < 1 or n_in < min_members:
        pos = rng.uniform(0.0, box, size=(3, n)).astype(np.float32)
        pos[pos >= np.float32(box)] = 0.0
        return pos
    # power-law weights by inverse transform on [1, 1000], then scaled to n_in members in total
    u = rng.uniform(size=n_halo)
    e = slope + 1.0
    w = (1.0 + u * (1000.0 ** e - 1.0)) ** (1.0 / e)
    m = np.maximum(min_members, np.floor(w / w.sum() * n_in)).astype(np.int64)
    while m.sum() > n_in and m.max() > min_members:
        m[np.argmax(m)] -= m.sum() - n_in if m.max() - (m.sum() - n_in) >= min_members else 1
    m = m[np.cumsum(m) <= n_in]
    n_in = int(m.sum())
    centres = rng.uniform(0.0, box, size=(3, len(m)))
    scale = halo_radius * (m / m.mean()) ** (1.0 / 3.0)
    owner = np.repeat(np.arange(len(m)), m)
    x = rng.uniform(size=n_in) * 0.98 + 0.01
    r = scale[owner] / np.sqrt(x ** (-2.0 / 3.0) - 1.0)  # Plummer enclosed-mass inverse
    r = np.minimum(r, 6.0 * scale[owner])
    v = rng.normal(size=(3, n_in))
    v /= np.linalg.norm(v, axis=0)
    pos = np.empty((3, n))
    pos[:, :n_in] = centres[:, owner] + v * r
    pos[:, n_in:] = rng.uniform(0.0, box, size=(3, n - n_in))
    pos = np.ascontiguousarray(np.mod(pos, box)[:, rng.permutation(n)], dtype=np.float32)
    pos[pos >= np.float32(box)] = 0.0
    return pos
