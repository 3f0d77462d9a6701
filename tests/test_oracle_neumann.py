"""Pins of the oracle's natural Neumann outflow boundary (Sec. 2:
du/dn = n p on the Neumann part of the boundary, Dirichlet elsewhere).

The outflow condition is natural (the weak form carries no boundary term),
so the oracle's only changes are which velocity DoFs are unknowns and the
absence of the pressure null space.  Pinned by: the unknown counts of the
face, a regular (full-rank, symmetric) coarse system where the all-Dirichlet
one has exactly one null vector, exact reproduction of fields inside the
element spaces that satisfy the outflow condition, and the discretisation
orders on a smooth manufactured solution (P1-P1: 2 / 2; P2-P1: 3 / 2.4,
the same as with Dirichlet data).  A planted mistake -- the face rows left
out, or the pressure shifted to zero mean -- breaks the reproduction.
"""
import numpy as np
import pytest

from oracle import coarse, fe, mesh, multigrid as mg
from oracle.stokes import Stokes
from paper_2010_13513_amd import workloads as W

NF = W.OUTFLOW_FACES


@pytest.mark.parametrize("vorder,N", [(1, 4), (2, 3)])
def test_outflow_face_unknowns(vorder, N):
    """Velocity unknowns = interior nodes + the nodes inside the face x = 1
    (not on its four Dirichlet edges): (M-1)^2 more per component."""
    M = vorder * N
    d = fe.Level(N, vorder)
    n = fe.Level(N, vorder, neumann=NF)
    assert d.vint.sum() == (M - 1) ** 3
    assert n.vint.sum() == (M - 1) ** 3 + (M - 1) ** 2
    c = n.vcoords
    extra = n.vint & ~d.vint
    assert np.all(c[extra, 0] == M) and np.all((c[extra, 1:] > 0) & (c[extra, 1:] < M))
    assert mesh.on_dirichlet(np.array([[M, 0, 3]]), M, NF)[0]          # edge with a Dirichlet face


@pytest.mark.parametrize("vorder,N", [(1, 2), (2, 2)])
def test_outflow_system_is_regular_and_symmetric(vorder, N):
    cd = coarse.CoarseSolver(Stokes(fe.Level(N, vorder)))
    cn = coarse.CoarseSolver(Stokes(fe.Level(N, vorder, neumann=NF)))
    assert cd.rank == cd.K.shape[0] - 1                 # (0, 1_p) with all-Dirichlet data
    assert cn.rank == cn.K.shape[0]
    assert np.abs(cn.K - cn.K.T).max() <= 1e-15 * np.abs(cn.K).max()


@pytest.mark.parametrize("vorder,lmin,L", [(1, 0, 2), (1, 1, 3), (2, 1, 2)])
def test_outflow_polynomial_reproduced(vorder, lmin, L):
    prob = W.outflow_polynomial(vorder)
    H = mg.Hierarchy(vorder, lmin, L, neumann=NF, schur="sd")
    xs = H.S[L].interpolate(prob.u, prob.p)
    x = H.exact_discrete(L, prob)
    assert np.abs(x - xs).max() < 1e-9
    # FMG with enough cycles gets there too (no mean-zero step anywhere)
    x = H.fmg(prob, mg.Params(2, 2, 0, 1, "f", 1 if vorder == 1 else 3, 2.3), cycles_on_finest=30)
    assert np.abs(x - xs).max() < 1e-8


def test_planted_mistakes_break_reproduction():
    """With the face rows treated as Dirichlet (the all-Dirichlet reading) or
    the pressure shifted to zero mean, the polynomial is not reproduced."""
    prob = W.outflow_polynomial(2)
    H = mg.Hierarchy(2, 1, 2, neumann=NF, schur="sd")
    xs = H.S[2].interpolate(prob.u, prob.p)
    Hd = mg.Hierarchy(2, 1, 2, schur="sd")
    xd = Hd.exact_discrete(2, prob, b=Hd.rhs(2, prob))
    assert np.abs(xd - xs).max() > 1e-2
    us, p = H.S[2].split(xs)
    m = H.S[2].lev.ML
    shifted = H.S[2].join(us, p - (m @ p) / m.sum())
    r = H.S[2].residual(shifted, H.rhs(2, prob))
    assert np.abs(r).max() > 1e-3
    assert np.abs(H.S[2].residual(xs, H.rhs(2, prob))).max() < 1e-12


@pytest.mark.slow
def test_outflow_discretisation_orders():
    """Smooth outflow solution (workloads.outflow_cube): errors of eq. error of
    the discrete solution fall at the optimal rates."""
    prob = W.outflow_cube()
    for vorder, Ls, want in ((1, (2, 3), (1.8, 1.8)), (2, (1, 2), (2.7, 2.7))):
        errs = []
        for L in Ls:
            H = mg.Hierarchy(vorder, 0 if vorder == 1 else 1, L + 1, neumann=NF, schur="sd")
            x = H.exact_discrete(L, prob)
            errs.append(mg.l2_errors(H.S[L + 1], H.T[L + 1], x, prob))
        rate = np.log2(np.array(errs[0]) / np.array(errs[1]))
        print(vorder, errs, rate)
        assert rate[0] > want[0] and rate[1] > want[1], (vorder, rate)
