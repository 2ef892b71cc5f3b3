"""Friends-of-friends haloes, their catalogue and the halo mass function (reference).

Test infrastructure only (see the package docstring).

Sec. 2.1 identifies haloes with the friends-of-friends algorithm of Davis et al. (1985) at a
linking length of 0.2 (read here, as is usual, in units of the mean inter-particle separation
L / N_p).  Sec. 2.5 keeps haloes of more than 100 particles and gives them the Warren et al. mass
M = m_p N (1 - N^-0.6).

Definition followed here.  Two particles are friends when their periodic distance is below the
linking length b; haloes are the connected components of the friendship graph; a group is
labelled by its smallest particle index.  Whether a pair are friends is an integer decision
taken from floating point, so it is made in float32 with every operation rounded on its own
(the precision the particle positions are stored in):

  d = x_j - x_i;  d -= L if d > L/2;  d += L if d < -L/2      (each axis, float32)
  d2 = (dx*dx + dy*dy) + dz*dz                                  (float32, no fused multiply-add)
  friends  iff  d2 < b2,   b2 = float32(b) * float32(b) rounded to float32.

Steps: candidate pairs from a k-d tree at a slightly larger float64 radius (a library
primitive), the exact float32 test above on each candidate, connected components of the
resulting graph (a library primitive), then labels, sizes, the catalogue and the binned mass
function, each written out below.

Catalogue: every group with N >= n_min, ordered by label, with N, the Warren mass and the centre
of mass: the label particle's position plus the mean of the float32 minimum-image offsets of
the members from it, wrapped into [0, L).
"""

import numpy as np
from scipy import sparse
from scipy.sparse import csgraph
from scipy.spatial import cKDTree

from .cosmology import warren_mass


def _f32(v):
    return np.float32(v)


def min_image_f32(d, box):
    """Per-axis minimum image of float32 differences, one correction of +-L."""
    box = _f32(box)
    half = _f32(0.5) * box
    d = np.asarray(d, dtype=np.float32)
    return np.where(d > half, d - box, np.where(d < -half, d + box, d)).astype(np.float32)


def pair_d2_f32(pos, i, j, box):
    """float32 squared periodic distance of the pairs (i[k], j[k]); pos: (3, n) float32."""
    dx = min_image_f32(pos[0, j] - pos[0, i], box)
    dy = min_image_f32(pos[1, j] - pos[1, i], box)
    dz = min_image_f32(pos[2, j] - pos[2, i], box)
    return (dx * dx + dy * dy) + dz * dz  # float32 arrays: each product and sum rounded once


def link2_f32(link):
    return _f32(link) * _f32(link)


def friend_pairs(pos, box, link):
    """All friend pairs (i < j) of float32 positions pos (3, n) in a periodic box."""
    pos = np.asarray(pos, dtype=np.float32)
    n = pos.shape[1]
    if n < 2:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    # the tree needs coordinates in [0, L): wrap a copy for the search only
    pts = np.mod(pos.T.astype(np.float64), box)
    pts[pts >= box] = 0.0
    tree = cKDTree(pts, boxsize=box)
    cand = tree.query_pairs(r=link * (1.0 + 1e-4) + 1e-6 * box, output_type="ndarray")
    if cand.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    i = np.minimum(cand[:, 0], cand[:, 1]).astype(np.int64)
    j = np.maximum(cand[:, 0], cand[:, 1]).astype(np.int64)
    keep = pair_d2_f32(pos, i, j, box) < link2_f32(link)
    return i[keep], j[keep]


def groups_from_pairs(n, i, j):
    """Labels (smallest member index) and per-label sizes of the components of the pair graph."""
    g = sparse.coo_matrix((np.ones(len(i), dtype=np.int8), (i, j)), shape=(n, n)).tocsr()
    _, comp = csgraph.connected_components(g, directed=False)
    label_of_comp = np.full(comp.max() + 1 if n else 0, n, dtype=np.int64)
    np.minimum.at(label_of_comp, comp, np.arange(n))
    group = label_of_comp[comp]
    size = np.zeros(n, dtype=np.int64)
    np.add.at(size, group, 1)
    return group.astype(np.int32), size.astype(np.int32)


def fof(pos, box, link):
    """(group, size): group[i] = smallest particle index of i's group; size[r] = members of the
    group labelled r (0 where r is no label)."""
    pos = np.asarray(pos, dtype=np.float32)
    i, j = friend_pairs(pos, box, link)
    return groups_from_pairs(pos.shape[1], i, j)


def linking_length(box, n_part, b=0.2):
    """b times the mean inter-particle separation L / N_p (Sec. 2.1)."""
    return b * box / n_part


def catalogue(pos, box, group, size, n_min, m_p):
    """Groups with at least n_min members, by increasing label: dict of arrays root, n, mass
    (Warren, Sec. 2.5) and com (3, n_halo) in [0, L)."""
    pos = np.asarray(pos, dtype=np.float32)
    roots = np.nonzero(size >= n_min)[0]
    n_h = size[roots].astype(np.int64)
    com = np.zeros((3, len(roots)))
    index = np.full(len(size), -1, dtype=np.int64)
    index[roots] = np.arange(len(roots))
    member = index[group] >= 0
    h = index[group[member]]
    idx = np.nonzero(member)[0]
    for d in range(3):
        off = min_image_f32(pos[d, idx] - pos[d, group[idx]], box).astype(np.float64)
        s = np.zeros(len(roots))
        np.add.at(s, h, off)
        c = pos[d, roots].astype(np.float64) + s / n_h
        c = np.where(c >= box, c - box, np.where(c < 0.0, c + box, c))
        com[d] = c
    return dict(root=roots.astype(np.int32), n=n_h.astype(np.int32), mass=warren_mass(n_h, m_p), com=com)


def mass_histogram(size, n_min, m_p, log10_edges):
    """Number of groups with N >= n_min whose Warren mass lies in [10^e_b, 10^e_{b+1})."""
    n_h = size[size >= n_min].astype(np.int64)
    m = warren_mass(n_h, m_p)
    edges = 10.0 ** np.asarray(log10_edges, dtype=np.float64)
    b = np.searchsorted(edges, m, side="right") - 1
    ok = (b >= 0) & (b < len(edges) - 1)
    return np.bincount(b[ok], minlength=len(edges) - 1).astype(np.int64)


def mass_function(counts, box, log10_edges):
    """dn / dlog10 M in (h^-1 Mpc)^-3 from binned counts in a box of side L."""
    return np.asarray(counts, dtype=np.float64) / (box ** 3 * np.diff(np.asarray(log10_edges, dtype=np.float64)))
