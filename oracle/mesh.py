"""Macro mesh, Bey refinement and the refined lattice (oracle; test infrastructure).

Paper Sec. 2 (uniform refinement of an unstructured macro mesh T_0 after Bey),
Sec. 2.1 (macro-primitives: every grid point belongs to exactly one of cell,
face, edge, vertex primitives), Sec. 2.2 (seven edge-DoF groups, eq.
num-unknowns-tet, Tab. unknown-count).

The macro mesh is the unit cube cut into the six Kuhn tetrahedra
conv{0, e_a, e_a+e_b, 1} (one per permutation (a,b,c)), vertices listed along
the Kuhn path.  Bey refinement of such a tetrahedron gives eight Kuhn
tetrahedra of half size, again in path order, so level l of the hierarchy is
the Freudenthal lattice with N = 2**(l + macro_refine) intervals per cube edge
(tested against an explicit Bey refinement in tests/test_oracle_mesh.py).

All coordinates here are integers in units of h = 1/N (P1 lattice) or h/2
(the doubled lattice that carries P2 nodes).
"""
from itertools import permutations

import numpy as np

PERMS = list(permutations(range(3)))          # fixed order of the 6 Kuhn types
E = np.eye(3, dtype=np.int64)

# Edge directions of the Freudenthal lattice, as parity classes of the doubled
# lattice; this is also the order of the edge colours 4..10.
EDGE_DIRS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]
P2_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]   # local P2 edge order


def kuhn_tet(origin, perm, scale=1):
    """Vertices of the Kuhn simplex at ``origin`` with step order ``perm``."""
    o = np.asarray(origin, dtype=np.int64)
    v0 = o
    v1 = v0 + scale * E[perm[0]]
    v2 = v1 + scale * E[perm[1]]
    v3 = o + scale * np.ones(3, dtype=np.int64)
    return np.stack([v0, v1, v2, v3])


def macro_mesh_cube():
    """The six Kuhn tetrahedra of the unit cube (integer coordinates)."""
    return [kuhn_tet((0, 0, 0), p) for p in PERMS]


def bey_refine(tets):
    """One step of Bey's red refinement (Sec. 2).

    Children of [x0,x1,x2,x3] with edge midpoints xij: the four corner
    tetrahedra and the octahedron cut along the x02-x13 diagonal, each child
    with Bey's vertex order.  Coordinates are doubled so they stay integer.
    """
    out = []
    for t in tets:
        x = [2 * np.asarray(v, dtype=np.int64) for v in t]
        m = {(i, j): (x[i] + x[j]) // 2 for i in range(4) for j in range(i + 1, 4)}
        out += [np.stack(c) for c in (
            (x[0], m[0, 1], m[0, 2], m[0, 3]),
            (m[0, 1], x[1], m[1, 2], m[1, 3]),
            (m[0, 2], m[1, 2], x[2], m[2, 3]),
            (m[0, 3], m[1, 3], m[2, 3], x[3]),
            (m[0, 1], m[0, 2], m[0, 3], m[1, 3]),
            (m[0, 1], m[0, 2], m[1, 2], m[1, 3]),
            (m[0, 2], m[0, 3], m[1, 3], m[2, 3]),
            (m[0, 2], m[1, 2], m[1, 3], m[2, 3]))]
    return out


def lattice_tets(N):
    """All tetrahedra of the level with N intervals: array (6*N^3, 4, 3).

    Ordered by Kuhn type (PERMS order), then cube index k, j, i.
    """
    g = np.arange(N)
    k, j, i = np.meshgrid(g, g, g, indexing="ij")
    org = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    tets = []
    for p in PERMS:
        t = kuhn_tet((0, 0, 0), p)
        tets.append(org[:, None, :] + t[None, :, :])
    return np.concatenate(tets, axis=0)


def n_tet(v):
    """eq. num-unknowns-tet: vertices of a refined tetrahedron with v per edge."""
    return (v + 2) * (v + 1) * v // 6


# ---------------------------------------------------------------------------
# Node numbering ("lattice order").  P1: (N+1)^3 nodes, index I + (N+1)(J +
# (N+1)K).  P2: doubled lattice (2N+1)^3, index X + (2N+1)(Y + (2N+1)Z).
# ---------------------------------------------------------------------------

def p1_index(N, I, J, K):
    n = N + 1
    return I + n * (J + n * K)


def p2_index(N, X, Y, Z):
    n = 2 * N + 1
    return X + n * (Y + n * Z)


def p1_coords(N):
    """(n^3, 3) integer coordinates of the P1 nodes in lattice order."""
    g = np.arange(N + 1)
    K, J, I = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)


def p2_coords(N):
    """(n^3, 3) doubled-lattice coordinates of the P2 nodes in lattice order."""
    g = np.arange(2 * N + 1)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def on_boundary(coords, M):
    """True where a node with integer coordinates in [0, M]^3 lies on the cube surface."""
    c = np.asarray(coords)
    return np.any((c == 0) | (c == M), axis=-1)


# Faces of the unit cube: 0: x = 0, 1: x = 1, 2: y = 0, 3: y = 1, 4: z = 0, 5: z = 1.
def on_dirichlet(coords, M, neumann=()):
    """True where a node lies on a face that is not in `neumann` (the Dirichlet
    part of the boundary is closed: a node on an edge or corner shared with a
    Dirichlet face is a Dirichlet node)."""
    c = np.asarray(coords)
    out = np.zeros(c.shape[:-1], dtype=bool)
    for f in range(6):
        if f in neumann:
            continue
        d, hi = f // 2, f % 2
        out |= c[..., d] == (M if hi else 0)
    return out


def p2_group(X, Y, Z):
    """DoF group of a doubled-lattice node: -1 vertex, else index into EDGE_DIRS."""
    par = (X % 2, Y % 2, Z % 2)
    if par == (0, 0, 0):
        return -1
    return EDGE_DIRS.index(par)


# ---------------------------------------------------------------------------
# Unknown counts per macro-cell and group (Tab. unknown-count).  The paper names
# the edge groups after the macro-cell's local index directions; for a Kuhn
# macro-cell conv{0, N e_a, N(e_a+e_b), N 1} the local directions x, y, z are
# e_a, e_a+e_b and (1,1,1), so the seven local groups correspond to global edge
# directions as below.
# ---------------------------------------------------------------------------

def local_group_dirs(perm):
    a, b, c = (E[p] for p in perm)
    one = np.ones(3, dtype=np.int64)
    return {"x": a, "y": a + b, "z": one, "xy": b, "xz": b + c, "yz": c, "xyz": a + c}


def _bary_int(tet, P):
    """Barycentric coordinates (times det) of doubled points P in doubled tet."""
    T = np.asarray(tet, dtype=np.int64)
    J = (T[1:] - T[0]).T.astype(float)
    lam = np.linalg.solve(J, (np.asarray(P, float) - T[0]).T).T
    lam0 = 1.0 - lam.sum(axis=1)
    return np.column_stack([lam0, lam])


def macro_cell_counts(N, perm):
    """Count vertex and edge nodes of each local group inside one macro-cell.

    Returns {group: (inner, including_boundary)} by brute-force point tests on
    the doubled lattice.
    """
    tet2 = 2 * kuhn_tet((0, 0, 0), perm, scale=N)
    pts = p2_coords(N)
    lam = _bary_int(tet2, pts)
    eps = 1e-9
    closed = np.all(lam > -eps, axis=1)
    inner = np.all(lam > eps, axis=1)
    par = pts % 2
    out = {}
    isv = np.all(par == 0, axis=1)
    out["vertex"] = (int(np.sum(inner & isv)), int(np.sum(closed & isv)))
    for name, d in local_group_dirs(perm).items():
        d = np.abs(d) % 2
        sel = np.all(par == d, axis=1)
        out[name] = (int(np.sum(inner & sel)), int(np.sum(closed & sel)))
    return out
