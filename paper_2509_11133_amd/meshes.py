"""Seeded synthetic inputs: initial meshes, coefficient fields and vertex jitter.

This module holds none of the method's arithmetic (no connectivity, refinement or FE
quantities): it only writes down level-0 meshes and draws random numbers on the host with
numpy's PCG64, so that the GPU library and the CPU oracle are fed identical arrays.

Layout: ``coord`` float64 (3, nC) and ``tet`` int32 (4, nE), 0-based, SoA (row k of the
array is column k of the paper's MATLAB matrices).  Boundary face lists are int32 (3, n).
"""
from __future__ import annotations

import numpy as np

JITTER_SEED = 2509
KAPPA_SEED = 11133

# Kuhn (Freudenthal) split of the unit cube into 6 tets along the main diagonal, written with
# the node numbering of the paper's initial mesh (Section 2.3: node 1+x+2y+4z at (x,y,z)).
# Rows follow the axis orders xyz, xzy, yxz, yzx, zxy, zyx; for the odd orders the last two
# vertices are swapped so that every tet has det[b-a, c-a, d-a] = +1 (one common sign is what
# the oriented-face connectivity of Section 3 needs).
_KUHN_1BASED = np.array([[1, 2, 4, 8], [1, 2, 8, 6], [1, 3, 8, 4], [1, 3, 7, 8], [1, 5, 6, 8], [1, 5, 8, 7]])


def _cube_coords():
    ids = np.arange(8)
    return np.stack([ids & 1, (ids >> 1) & 1, (ids >> 2) & 1]).astype(np.float64)


def kuhn_cube():
    """Unit cube, 8 nodes, 6 Kuhn tets.  Returns (coord, tet)."""
    return _cube_coords(), np.ascontiguousarray((_KUHN_1BASED - 1).T, dtype=np.int32)


def paper_cube():
    """The paper's initial mesh (Section 2.3): 5 tets, 2 Dirichlet and 10 Neumann faces.
    Returns (coord, tet, Db, Nb), 0-based."""
    coord = _cube_coords()
    tet = np.array([[1, 2, 3, 5], [5, 8, 6, 2], [7, 3, 8, 5], [4, 8, 3, 2], [8, 3, 2, 5]]) - 1
    db = np.array([[7, 8, 5], [5, 8, 6]]) - 1
    nb = np.array([[1, 5, 2], [5, 6, 2], [1, 3, 5], [7, 5, 3], [7, 3, 8], [4, 8, 3], [2, 6, 8], [4, 2, 8],
                   [4, 3, 2], [1, 2, 3]]) - 1
    as_soa = lambda a: np.ascontiguousarray(a.T, dtype=np.int32)
    return coord, as_soa(tet), as_soa(db), as_soa(nb)


def fichera():
    """Fichera-type domain: the 2x2x2 cube minus the octant [1,2]^3 (7 unit cubes x 6 Kuhn
    tets = 42 tets, 26 nodes).  Node id x + 3y + 9z on the grid {0,1,2}^3 without (2,2,2);
    cubes ordered z-major, x-minor.  Returns (coord, tet)."""
    g = np.arange(27)
    xyz = np.stack([g % 3, (g // 3) % 3, g // 9])[:, :26].astype(np.float64)
    loc = _KUHN_1BASED - 1  # local ids 0..7 = x + 2y + 4z
    lx, ly, lz = loc & 1, (loc >> 1) & 1, (loc >> 2) & 1
    tets = []
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                if (ox, oy, oz) == (1, 1, 1):
                    continue
                tets.append((ox + lx) + 3 * (oy + ly) + 9 * (oz + lz))
    tet = np.concatenate(tets, axis=0)
    return xyz, np.ascontiguousarray(tet.T, dtype=np.int32)


def boundary_faces_box(coord, tet, lo=0.0, hi=1.0):
    """Tet faces lying on the boundary of the box [lo,hi]^3, each as it occurs in its tet
    (local faces [a b c], [a c d], [a d b], [d c b]).  Used only to hand a level-0 Dirichlet
    list to the refinement; it classifies faces by coordinates, not by connectivity."""
    local = [(0, 1, 2), (0, 2, 3), (0, 3, 1), (3, 2, 1)]
    out = []
    for t in range(tet.shape[1]):
        for f in local:
            nodes = tet[list(f), t]
            p = coord[:, nodes]
            for d in range(3):
                if np.all(p[d] == lo) or np.all(p[d] == hi):
                    out.append(nodes)
                    break
    return np.ascontiguousarray(np.array(out, dtype=np.int32).T)


def min_edge_length(coord, tet):
    """Smallest tet edge length (the h of the jitter recipe), from the 6 edges of every tet."""
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    h = np.inf
    for a, b in pairs:
        d = coord[:, tet[a]] - coord[:, tet[b]]
        h = min(h, float(np.sqrt((d * d).sum(axis=0)).min()))
    return h


def jitter_unit_cube(coord, tet, frac=0.1, seed=JITTER_SEED):
    """Move every vertex strictly inside the unit cube by U[-frac h, frac h] per coordinate,
    h = smallest edge length of the mesh.  Boundary vertices stay put."""
    h = min_edge_length(coord, tet)
    rng = np.random.Generator(np.random.PCG64(seed))
    inside = np.all((coord > 0.0) & (coord < 1.0), axis=0)
    out = coord.copy()
    delta = rng.uniform(-frac * h, frac * h, size=(3, int(inside.sum())))
    out[:, inside] += delta
    return out


def lognormal_kappa(nE, sigma=1.0, seed=KAPPA_SEED):
    """kappa_T = exp(sigma g_T), g_T ~ N(0,1) i.i.d. per tet."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(sigma * rng.standard_normal(nE))


def lognormal_kappa_fields(nE, nk, sigma=1.0, seed=KAPPA_SEED):
    """nk independent lognormal fields [nk, nE] (field j seeded with seed + j)."""
    return np.stack([lognormal_kappa(nE, sigma, seed + j) for j in range(nk)])


SIN3_AMPLITUDE = 3.0 * np.pi ** 2 + 1.0  # f = (3 pi^2 kappa + c) sin sin sin for kappa = c = 1
