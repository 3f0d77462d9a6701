"""P1 / P2 finite elements and global assembly (oracle; test infrastructure).

Paper Sec. 2, eq. stokes-weak / stokes-discrete: a_ij = int grad phi_i : grad
phi_j, b_kj = -int psi_k div phi_j; eq. pspg: c_ij = sum_T delta_T h_T^2 int_T
grad psi_i . grad psi_j with h_T = |T|^(1/3), delta_T = 1/12.

Basis functions are polynomials in the four barycentric coordinates
(dict exponent-tuple -> coefficient).  Integrals use the exact formula
int_T lam^alpha dx = 6|T| alpha! / (|alpha| + 3)!.

Boundary (Sec. 2): Dirichlet on the faces of the cube not listed in
`neumann`, natural Neumann outflow (du/dn = n p) on the listed ones.  The
outflow condition is natural: the weak form has no boundary term, so the
velocity DoFs on a Neumann face (not on its Dirichlet edges) are unknowns with
the assembled rows of A and B^T, and the pressure has no null space.

Variable viscosity (not in the paper's experiments): the A block becomes
sum_T nu_T int_T grad phi_i . grad phi_j with nu_T the mean of nu at the four
vertices of T (per velocity component, so A stays block diagonal).
"""
from math import factorial

import numpy as np
import scipy.sparse as sp

from . import mesh

DELTA_PSPG = 1.0 / 12.0


# ----------------------------------------------------------------- polynomials
def _mono(idx, c=1.0):
    e = [0, 0, 0, 0]
    for i in idx:
        e[i] += 1
    return {tuple(e): c}


def _padd(p, q, s=1.0):
    r = dict(p)
    for k, v in q.items():
        r[k] = r.get(k, 0.0) + s * v
    return r


def _pmul(p, q):
    r = {}
    for k1, v1 in p.items():
        for k2, v2 in q.items():
            k = tuple(a + b for a, b in zip(k1, k2))
            r[k] = r.get(k, 0.0) + v1 * v2
    return r


def _pdiff(p, m):
    r = {}
    for k, v in p.items():
        if k[m] > 0:
            kk = list(k)
            kk[m] -= 1
            kk = tuple(kk)
            r[kk] = r.get(kk, 0.0) + v * k[m]
    return r


def _pint(p, vol):
    tot = 0.0
    for k, v in p.items():
        num = 1
        for a in k:
            num *= factorial(a)
        tot += v * 6.0 * vol * num / factorial(sum(k) + 3)
    return tot


def basis(order):
    """Barycentric basis: P1 = lam_i; P2 = lam_i(2 lam_i - 1) then 4 lam_i lam_j."""
    if order == 1:
        return [_mono([i]) for i in range(4)]
    b = [_padd(_mono([i, i], 2.0), _mono([i]), -1.0) for i in range(4)]
    b += [_mono([i, j], 4.0) for (i, j) in mesh.P2_EDGES]
    return b


# -------------------------------------------------------------- element level
def geometry(X):
    """Volume and barycentric gradients (4, 3) of the tetrahedron X (4, 3)."""
    X = np.asarray(X, dtype=float)
    J = (X[1:] - X[0]).T
    vol = abs(np.linalg.det(J)) / 6.0
    Ji = np.linalg.inv(J)
    g = np.zeros((4, 3))
    g[1:] = Ji
    g[0] = -Ji.sum(axis=0)
    return vol, g


def local_stiffness(X, order):
    vol, g = geometry(X)
    G = g @ g.T
    b = basis(order)
    db = [[_pdiff(phi, m) for m in range(4)] for phi in b]
    n = len(b)
    K = np.zeros((n, n))
    for a in range(n):
        for c in range(n):
            s = 0.0
            for m in range(4):
                for q in range(4):
                    if G[m, q] != 0.0:
                        s += G[m, q] * _pint(_pmul(db[a][m], db[c][q]), vol)
            K[a, c] = s
    return K


def local_mass(X, order):
    vol, _ = geometry(X)
    b = basis(order)
    return np.array([[_pint(_pmul(p, q), vol) for q in b] for p in b])


def local_load(X, order):
    vol, _ = geometry(X)
    return np.array([_pint(p, vol) for p in basis(order)])


def local_divergence(X, vorder):
    """D[d, k, a] = -int psi_k d/dx_d phi_a, psi P1 (pressure), phi of order vorder."""
    vol, g = geometry(X)
    psi = basis(1)
    phi = basis(vorder)
    D = np.zeros((3, 4, len(phi)))
    for a, p in enumerate(phi):
        dp = [_pdiff(p, m) for m in range(4)]
        for k in range(4):
            ints = np.array([_pint(_pmul(psi[k], dp[m]), vol) for m in range(4)])
            D[:, k, a] = -(g.T @ ints)
    return D


def local_pspg(X):
    vol, _ = geometry(X)
    h2 = vol ** (2.0 / 3.0)
    return DELTA_PSPG * h2 * local_stiffness(X, 1)


# ------------------------------------------------------------------- assembly
def element_dofs(tets, N, order):
    """Global DoF indices (lattice order) of each element: (ne, 4) or (ne, 10)."""
    t = np.asarray(tets, dtype=np.int64)
    if order == 1:
        return mesh.p1_index(N, t[..., 0], t[..., 1], t[..., 2])
    cols = [2 * t[:, i, :] for i in range(4)]
    cols += [t[:, i, :] + t[:, j, :] for (i, j) in mesh.P2_EDGES]
    P = np.stack(cols, axis=1)
    return mesh.p2_index(N, P[..., 0], P[..., 1], P[..., 2])


class Level:
    """Assembled float64 operators of one level of the Kuhn-cube hierarchy.

    vorder = 1 (P1-P1 PSPG) or 2 (P2-P1 Taylor-Hood).  nu_vertex: optional
    viscosity at the P1 nodes (lattice order) for the variable-viscosity A.
    neumann: faces (mesh.on_dirichlet numbering) with the outflow condition.
    """

    def __init__(self, N, vorder, nu_vertex=None, neumann=()):
        self.N = N
        self.vorder = vorder
        self.h = 1.0 / N
        tets = mesh.lattice_tets(N)
        self.tets = tets
        ne = tets.shape[0]
        nper = N ** 3
        self.np_ = (N + 1) ** 3
        self.nv = self.np_ if vorder == 1 else (2 * N + 1) ** 3
        vd = element_dofs(tets, N, vorder)
        pd = element_dofs(tets, N, 1)
        self.vdofs, self.pdofs = vd, pd
        h = self.h
        nloc = vd.shape[1]
        Ks, Ms, Ds, Cs, Mps, loads = [], [], [], [], [], []
        for p in mesh.PERMS:
            X = mesh.kuhn_tet((0, 0, 0), p) * h
            Ks.append(local_stiffness(X, vorder))
            Ms.append(local_mass(X, vorder))
            Ds.append(local_divergence(X, vorder))
            Cs.append(local_pspg(X))
            Mps.append(local_mass(X, 1))
            loads.append(local_load(X, 1))
        typ = np.repeat(np.arange(6), nper)
        K = np.stack(Ks)[typ]                   # (ne, nloc, nloc)
        if nu_vertex is not None:
            nuT = np.asarray(nu_vertex)[pd].mean(axis=1)
            K = K * nuT[:, None, None]
            self.nu_elem = nuT
        M = np.stack(Ms)[typ]
        D = np.stack(Ds)[typ]                   # (ne, 3, 4, nloc)
        C = np.stack(Cs)[typ]
        Mp = np.stack(Mps)[typ]
        ld = np.stack(loads)[typ]

        def asm(loc, rows, cols, n, m):
            r = np.repeat(rows[:, :, None], cols.shape[1], axis=2)
            c = np.repeat(cols[:, None, :], rows.shape[1], axis=1)
            return sp.csr_matrix((loc.ravel(), (r.ravel(), c.ravel())), shape=(n, m))

        self.A = asm(K, vd, vd, self.nv, self.nv)
        self.M = asm(M, vd, vd, self.nv, self.nv)
        self.B = [asm(D[:, d], pd, vd, self.np_, self.nv) for d in range(3)]
        self.C = asm(C, pd, pd, self.np_, self.np_)
        if vorder == 2:
            self.C = sp.csr_matrix((self.np_, self.np_))   # Taylor-Hood: C = 0
        self.Mp = asm(Mp, pd, pd, self.np_, self.np_)
        ml = np.zeros(self.np_)
        np.add.at(ml, pd.ravel(), ld.ravel())
        self.ML = ml                         # lumped P1 mass (diagonal) = int psi_k
        vc = mesh.p1_coords(N) if vorder == 1 else mesh.p2_coords(N)
        self.vcoords = vc                    # integer coords, units h / vorder
        self.pcoords = mesh.p1_coords(N)
        self.neumann = tuple(sorted(set(neumann)))
        self.vbnd = mesh.on_dirichlet(vc, N * vorder, self.neumann)   # Dirichlet velocity nodes
        self.vint = ~self.vbnd                                         # velocity unknowns
        self.Adiag = self.A.diagonal()

    # positions in [0,1]^3
    def vpos(self):
        return self.vcoords / float(self.N * self.vorder)

    def ppos(self):
        return self.pcoords / float(self.N)
