"""Unstructured macro meshes (oracle; test infrastructure).

Paper Sec. 2 / 2.1: an unstructured partition T_0 of the domain into
tetrahedra is refined uniformly (Bey's red refinement) L times; every refined
node belongs to exactly one macro-primitive (vertex, edge, face or cell of
T_0).  Here for the P1-P1 PSPG discretisation (eq. pspg) on any T_0.

Nodes are identified exactly by their barycentric weights in a macro cell:
a level-l node of macro cell (v_0 < v_1 < v_2 < v_3) (vertex ids sorted, so
that two cells induce the same refinement on a shared face or edge) has
integer weights a_k >= 0 with sum n = 2^l; its key is ((v_k, a_k) for a_k >
0), the same from every cell that contains it.  The macro-primitive of the
node is the set of v_k with a_k > 0.

Canonical node order (the order of every vector here): by primitive
dimension (vertices, edges, faces, cells), then by the sorted vertex ids of
the primitive, then by the weight tuple (in vertex-id order).

Refinement follows Bey's rule (mesh.bey_refine) applied to the barycentric
coordinates, which also gives the linear prolongation: every node of level
l + 1 is a node of level l or the midpoint of an edge of a level-l element.

Element matrices are the closed forms of P1 elements (gradients constant):
stiffness |T| G G^T, consistent mass |T| (1 + delta_ij) / 20, divergence
b_kj = -(|T| / 4) d phi_j / dx_d, PSPG delta |T|^(2/3) x stiffness, lumped
mass |T| / 4 per vertex (tests check them against fe.local_*).

Boundary: Dirichlet on the faces of T_0 that belong to one cell only.

Gauss-Seidel colouring: nodes on vertices, edges and faces of T_0 are
coloured greedily in canonical order (the smallest colour not used by a
coupled, i.e. element-sharing, node that comes earlier); the interior nodes
of the cells take K + ((a_1 + 2 a_2 + 3 a_3) mod 4), K the number of greedy
colours -- conflict-free because two interior nodes of a cell that share an
element differ by one of the 14 lattice offsets of the refined cell, whose
weighted sums are 1, 2 or 3 (mod 4, never 0).
"""
import numpy as np
import scipy.sparse as sp

from . import fe, mesh
from .transfer import Transfer


def boundary_faces(tets):
    """Faces (sorted vertex triples) of T_0 that belong to one tetrahedron."""
    count = {}
    for t in tets:
        for drop in range(4):
            f = tuple(sorted(int(v) for q, v in enumerate(t) if q != drop))
            count[f] = count.get(f, 0) + 1
    return {f for f, c in count.items() if c == 1}


def p1_closed_forms(X):
    """(stiffness, mass, divergence (3, 4, 4), lumped mass) of the P1 element X."""
    vol, g = fe.geometry(X)
    K = vol * g @ g.T
    M = vol / 20.0 * (np.ones((4, 4)) + np.eye(4))
    D = np.zeros((3, 4, 4))
    for d in range(3):
        D[d] = -(vol / 4.0) * np.tile(g[:, d], (4, 1))     # row k (pressure), col j (velocity)
    return vol, K, M, D


class ULevel:
    """Assembled P1-P1 PSPG operators of level l of an unstructured T_0,
    with the attributes of fe.Level that the Stokes, smoother, coarse-solve
    and multigrid code reads."""

    def __init__(self, xyz, tets, level, bfaces=None, outflow=()):
        """outflow: boundary faces (vertex triples) with the natural outflow
        condition (Sec. 2, du/dn = n p); the other boundary faces are
        Dirichlet, their closure included."""
        self.vorder = 1
        self.N = 2 ** level
        outflow = {tuple(sorted(int(v) for v in f)) for f in outflow}
        self.neumann = tuple(sorted(outflow))
        n = self.N
        xyz = np.asarray(xyz, dtype=float)
        self.tets0 = [tuple(sorted(int(v) for v in t)) for t in tets]
        bfaces = boundary_faces(tets) if bfaces is None else bfaces
        assert outflow <= set(bfaces), "outflow faces must be boundary faces"
        bfaces = set(bfaces) - outflow          # the Dirichlet faces
        # refined elements of every macro cell, in barycentric weights (sum n)
        keyset = {}
        elems = []           # (cell index, 4 keys)
        self.parents = {}    # key -> (parent key, parent key) of the level below (midpoints)
        for c, tv in enumerate(self.tets0):
            els = [np.eye(4, dtype=np.int64)]          # level 0: the cell itself
            for _ in range(level):
                els = mesh.bey_refine(els)
            for e in els:
                ks = [self._key(tv, a) for a in e]
                elems.append((c, ks, e))
                for k in ks:
                    keyset[k] = True
        keys = sorted(keyset, key=self._order)
        self.keys = keys
        self.index = {k: q for q, k in enumerate(keys)}
        nn = len(keys)
        self.np_ = self.nv = nn
        # positions
        pos = np.zeros((nn, 3))
        for k, q in self.index.items():
            pos[q] = sum(a * xyz[v] for v, a in k) / n
        self._pos = pos
        # assembly
        rows, cols, A, M, C, Ml = [], [], [], [], [], np.zeros(nn)
        Bv = [[], [], []]
        for c, ks, _ in elems:
            X = pos[[self.index[k] for k in ks]]
            vol, K, Me, D = p1_closed_forms(X)
            ids = np.array([self.index[k] for k in ks])
            rows.append(np.repeat(ids, 4))
            cols.append(np.tile(ids, 4))
            A.append(K.ravel())
            M.append(Me.ravel())
            C.append((fe.DELTA_PSPG * vol ** (2.0 / 3.0) * K).ravel())
            for d in range(3):
                Bv[d].append(D[d].ravel())
            np.add.at(Ml, ids, vol / 4.0)
        r, cc = np.concatenate(rows), np.concatenate(cols)
        mk = lambda v: sp.csr_matrix((np.concatenate(v), (r, cc)), shape=(nn, nn))
        self.A = mk(A)
        self.M = mk(M)
        self.Mp = self.M
        self.C = mk(C)
        self.B = [mk(Bv[d]) for d in range(3)]
        self.ML = Ml
        self.Adiag = self.A.diagonal()
        # Dirichlet nodes: on a boundary face of T_0
        self.vbnd = np.array([any(set(v for v, _ in k) <= set(f) for f in bfaces) for k in keys])
        self.vint = ~self.vbnd
        # coupling pattern (nodes sharing an element) and the colouring
        self.elem_ids = np.array([[self.index[k] for k in ks] for _, ks, _ in elems])
        self.elem_cell = np.array([c for c, _, _ in elems])
        self.colour, self.ncolours = self._colouring()

    # ------------------------------------------------------------------ keys
    @staticmethod
    def _key(tv, a):
        return tuple((int(v), int(x)) for v, x in zip(tv, a) if x > 0)

    @staticmethod
    def _order(k):
        return (len(k), tuple(v for v, _ in k), tuple(x for _, x in k))

    def _colouring(self):
        nn = self.nv
        dim = np.array([len(k) for k in self.keys])
        nbr = [set() for _ in range(nn)]
        for e in self.elem_ids:
            for a in e:
                for b in e:
                    if a != b:
                        nbr[a].add(b)
        col = np.full(nn, -1, dtype=np.int64)
        iface = np.nonzero(dim < 4)[0]
        for q in iface:                       # canonical order
            used = {col[j] for j in nbr[q] if col[j] >= 0}
            c = 0
            while c in used:
                c += 1
            col[q] = c
        K = int(col[iface].max()) + 1 if iface.size else 0
        for q in np.nonzero(dim == 4)[0]:
            w = [x for _, x in self.keys[q]]         # a_0 .. a_3 in vertex-id order
            col[q] = K + (w[1] + 2 * w[2] + 3 * w[3]) % 4
        return col, K + 4

    # ------------------------------------------------------- fe.Level API
    def vpos(self):
        return self._pos

    def ppos(self):
        return self._pos


def prolongation(coarse, fine):
    """Linear interpolation from level l (coarse) to l + 1 (fine): a fine node
    that is a coarse node takes its value, a midpoint of a coarse element edge
    the mean of the edge's ends (found by refining the coarse elements once)."""
    P = sp.lil_matrix((fine.nv, coarse.nv))
    done = np.zeros(fine.nv, dtype=bool)
    # refine every coarse element once; Bey's children have the parent's
    # vertices and the edge midpoints as vertices
    for e_ids, cell in zip(coarse.elem_ids, coarse.elem_cell):
        tv = coarse.tets0[cell]
        keys = [coarse.keys[q] for q in e_ids]
        bary = [np.zeros(4, dtype=np.int64) for _ in keys]
        for b, k in zip(bary, keys):
            for v, a in k:
                b[tv.index(v)] = a
        for i in range(4):
            kf = ULevel._key(tv, 2 * bary[i])
            q = fine.index[kf]
            if not done[q]:
                P[q, e_ids[i]] = 1.0
                done[q] = True
            for j in range(i + 1, 4):
                kf = ULevel._key(tv, bary[i] + bary[j])
                q = fine.index[kf]
                if not done[q]:
                    P[q, e_ids[i]] = 0.5
                    P[q, e_ids[j]] = 0.5
                    done[q] = True
    assert done.all()
    return P.tocsr()


class UTransfer(Transfer):
    """Prolongation / restriction of Stokes vectors between two levels of an
    unstructured hierarchy: the linear interpolation of `prolongation` for
    velocity and pressure alike (Sec. 3.3), restriction its transpose."""

    def __init__(self, Sc, Sf):
        self.Sc, self.Sf = Sc, Sf
        P = prolongation(Sc.lev, Sf.lev)
        self.Pv = self.Pp = P
        self.Rv = self.Rp = P.T.tocsr()


def hierarchy(xyz, tets, Lmin, Lmax, schur="ml", outflow=()):
    """multigrid.Hierarchy on the levels Lmin..Lmax of T_0 = (xyz, tets),
    `outflow` boundary faces with the natural outflow condition."""
    from . import multigrid as mg
    from .coarse import CoarseSolver
    from .smoother import Uzawa
    from .stokes import Stokes
    H = mg.Hierarchy.__new__(mg.Hierarchy)
    H.vorder, H.Lmin, H.Lmax, H.mr, H.nu_fn = 1, Lmin, Lmax, 0, None
    H.neumann = tuple(sorted(tuple(sorted(int(v) for v in f)) for f in outflow))
    H.S, H.U, H.T = {}, {}, {}
    bf = boundary_faces(tets)
    for l in range(Lmin, Lmax + 1):
        H.S[l] = Stokes(ULevel(xyz, tets, l, bf, outflow))
        H.U[l] = Uzawa(H.S[l], schur)
    for l in range(Lmin + 1, Lmax + 1):
        H.T[l] = UTransfer(H.S[l - 1], H.S[l])
    H.coarse = CoarseSolver(H.S[Lmin])
    return H
