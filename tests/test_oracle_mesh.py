"""Pins of the oracle's mesh and counting code (Sec. 2, 2.1, 2.2)."""
import numpy as np
import pytest

from oracle import fe, mesh


def _as_set(tets):
    return {tuple(map(tuple, np.asarray(t).tolist())) for t in tets}


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_bey_refinement_gives_freudenthal_lattice(levels):
    """Bey refinement (explicit rule) of the six Kuhn tetrahedra equals the
    lattice tetrahedra with N = 2**levels, vertex order included."""
    tets = mesh.macro_mesh_cube()
    for _ in range(levels):
        tets = mesh.bey_refine(tets)
    assert len(tets) == 6 * 8 ** levels
    assert _as_set(tets) == _as_set(mesh.lattice_tets(2 ** levels))


def test_48_tet_macro_mesh_is_one_bey_step():
    t48 = mesh.bey_refine(mesh.macro_mesh_cube())
    assert len(t48) == 48
    # refining the 48-tet mesh l times gives the lattice with 2**(l+1) intervals
    assert _as_set(mesh.bey_refine(t48)) == _as_set(mesh.lattice_tets(4))


def test_lattice_volumes_partition_cube():
    N = 3
    tets = mesh.lattice_tets(N).astype(float) / N
    vols = [fe.geometry(t)[0] for t in tets]
    assert np.allclose(vols, 1.0 / (6 * N ** 3), rtol=0, atol=1e-15)
    assert abs(sum(vols) - 1.0) < 1e-13


def test_bey_children_are_congruent_classes():
    """Sec. 2.1: refined tetrahedra fall into few congruence classes; on the
    Kuhn cube all children are Kuhn simplices (one of the six step orders)."""
    tets = mesh.bey_refine(mesh.bey_refine(mesh.macro_mesh_cube()))
    for t in tets:
        steps = np.diff(np.asarray(t), axis=0)
        assert sorted(map(tuple, steps.tolist())) == [(0, 0, 1), (0, 1, 0), (1, 0, 0)]


def test_n_tet_closed_form():
    # eq. num-unknowns-tet: tetrahedral numbers
    assert [mesh.n_tet(v) for v in range(1, 7)] == [1, 4, 10, 20, 35, 56]


@pytest.mark.parametrize("level", [2, 3, 4])
@pytest.mark.parametrize("perm", mesh.PERMS)
def test_unknown_count_table(level, perm):
    """Tab. unknown-count by brute-force point counting in one macro-cell."""
    n = 2 ** level
    cnt = mesh.macro_cell_counts(n, perm)
    nt = mesh.n_tet
    assert cnt["vertex"] == (nt(n - 3), nt(n + 1))
    assert cnt["xyz"] == (nt(n - 1), nt(n - 1))
    for g in ("x", "y", "z", "xy", "xz", "yz"):
        assert cnt[g] == (nt(n - 2), nt(n)), g


@pytest.mark.parametrize("N", [1, 2, 4, 8])
def test_p2_unknowns_equal_p1_unknowns_next_level(N):
    """Sec. 2.2: P2 DoFs on level l equal P1 DoFs on level l+1."""
    assert mesh.p2_coords(N).shape[0] == mesh.p1_coords(2 * N).shape[0]


def test_stencil_count_table():
    """Tab. stencil-count: structural entries of the assembled P2 stiffness at
    interior nodes, all and vertex-only, per stencil centre."""
    rows = {}
    for line in open(__file__.replace("test_oracle_mesh.py", "golden/stencil_count.txt")):
        if line.strip() and not line.startswith("#"):
            name, fv, fa = line.split()
            rows[name] = (int(fv), int(fa))
    N = 4
    lev = fe.Level(N, 2)
    A = lev.A.tocsr()
    coords = lev.vcoords
    got = {}
    for par in [(0, 0, 0)] + mesh.EDGE_DIRS:
        X, Y, Z = (4 + p for p in par)
        r = A.indptr[mesh.p2_index(N, X, Y, Z)]
        r1 = A.indptr[mesh.p2_index(N, X, Y, Z) + 1]
        cols = A.indices[r:r1]
        nvert = int(np.sum(np.all(coords[cols] % 2 == 0, axis=1)))
        got[par] = (nvert, len(cols))
    assert got[(0, 0, 0)] == rows["vertex"]
    for perm in mesh.PERMS:
        for name, d in mesh.local_group_dirs(perm).items():
            assert got[tuple(int(v) for v in d)] == rows[name], (perm, name)
    # P1-P1: the 15-point stencil (vertex row of the table)
    l1 = fe.Level(4, 1)
    i = mesh.p1_index(4, 2, 2, 2)
    assert l1.A.indptr[i + 1] - l1.A.indptr[i] == rows["vertex"][0]
