"""Pins of the oracle's finite-element operators (eq. stokes-discrete, eq. pspg).

Each check compares with something the oracle does not compute itself:
closed-form stencils, exact polynomial integrals, textbook identities.
"""
import numpy as np
import pytest

from oracle import fe, mesh


def _poly_vals(c, q):
    return q(c[:, 0], c[:, 1], c[:, 2])


def test_p1_stiffness_is_seven_point_laplacian():
    """On the Kuhn lattice the P1 stiffness row is h * (6, -1 x 6)."""
    N = 5
    lev = fe.Level(N, 1)
    u = np.random.default_rng(1).standard_normal(lev.nv)
    Au = lev.A @ u
    U = u.reshape(N + 1, N + 1, N + 1)      # [K, J, I]
    lap = 6 * U[1:-1, 1:-1, 1:-1] - (U[:-2, 1:-1, 1:-1] + U[2:, 1:-1, 1:-1] + U[1:-1, :-2, 1:-1]
                                     + U[1:-1, 2:, 1:-1] + U[1:-1, 1:-1, :-2] + U[1:-1, 1:-1, 2:])
    got = Au.reshape(N + 1, N + 1, N + 1)[1:-1, 1:-1, 1:-1]
    want = lap / N
    assert np.allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_pspg_is_scaled_laplacian():
    """eq. pspg with h_T = |T|^(1/3) = (h^3/6)^(1/3), delta = 1/12: interior C
    rows are delta h_T^2 times the stiffness row."""
    N = 4
    lev = fe.Level(N, 1)
    hT2 = (1.0 / (6 * N ** 3)) ** (2.0 / 3.0)
    diff = (lev.C - lev.A * (hT2 / 12.0)).tocsr()
    assert abs(diff).max() < 1e-15


@pytest.mark.parametrize("vorder", [1, 2])
def test_symmetry_and_row_sums(vorder):
    lev = fe.Level(3, vorder)
    for Mx in (lev.A, lev.C, lev.M, lev.Mp):
        assert abs(Mx - Mx.T).max() < 1e-15
    one_v = np.ones(lev.nv)
    one_p = np.ones(lev.np_)
    assert np.abs(lev.A @ one_v).max() < 1e-13          # grad 1 = 0
    assert np.abs(lev.C @ one_p).max() < 1e-15
    for d in range(3):
        assert np.abs(lev.B[d] @ one_v).max() < 1e-14      # div(const) = 0
        bt1 = lev.B[d].T @ one_p                          # int div phi_j = 0 inside
        assert np.abs(bt1[lev.vint]).max() < 1e-14
        assert np.abs(bt1[lev.vbnd]).max() > 1e-3


@pytest.mark.parametrize("vorder", [1, 2])
def test_mass_integrates_polynomials(vorder):
    """1^T M I(q) = int_cube q for q in the element space (closed forms)."""
    N = 3
    lev = fe.Level(N, vorder)
    c = lev.vpos()
    if vorder == 1:
        q = lambda x, y, z: 1 + 2 * x - 3 * y + 0.5 * z      # integral 1 + 1 - 1.5 + 0.25
        exact = 1 + 1 - 1.5 + 0.25
    else:
        q = lambda x, y, z: x * y + z * z - 2 * x             # 1/4 + 1/3 - 1
        exact = 0.25 + 1.0 / 3.0 - 1.0
    assert abs(np.ones(lev.nv) @ (lev.M @ _poly_vals(c, q)) - exact) < 1e-13
    assert abs(lev.ML.sum() - 1.0) < 1e-13
    # consistent P1 mass: interior row sums are h^3
    l1 = fe.Level(N, 1)
    rs = l1.Mp @ np.ones(l1.np_)
    i = mesh.p1_index(N, 1, 1, 1)
    assert abs(rs[i] - N ** -3) < 1e-16


def test_patch_laplacian_quadratic():
    """P2: interior rows of A I(q) equal int (-lap q) phi_i = (-lap q) (M 1)_i
    for quadratic q; P1: A I(q) = 0 in interior rows for linear q."""
    N = 3
    lev = fe.Level(N, 2)
    c = lev.vpos()
    q = lambda x, y, z: 3 * x * x - y * z + 2 * y * y + x - 1    # lap q = 6 + 4 = 10
    Aq = lev.A @ _poly_vals(c, q)
    M1 = lev.M @ np.ones(lev.nv)
    assert np.allclose(Aq[lev.vint], -10.0 * M1[lev.vint], rtol=0, atol=1e-13)
    l1 = fe.Level(N, 1)
    c1 = l1.vpos()
    lin = lambda x, y, z: 2 * x - y + 3 * z + 1
    assert np.abs((l1.A @ _poly_vals(c1, lin))[l1.vint]).max() < 1e-14


def test_patch_divergence_taylor_hood():
    """B I(v) = -M_p I(div v) on all pressure rows for quadratic v (P2-P1)."""
    N = 3
    lev = fe.Level(N, 2)
    c = lev.vpos()
    v = [lambda x, y, z: x * x + y * z, lambda x, y, z: x * y - 2 * y * y, lambda x, y, z: z * x + y]
    div = lambda x, y, z: 2 * x + x - 4 * y + x      # d/dx v1 + d/dy v2 + d/dz v3
    Bv = sum(lev.B[d] @ _poly_vals(c, v[d]) for d in range(3))
    cp = lev.ppos()
    assert np.allclose(Bv, -(lev.Mp @ _poly_vals(cp, div)), rtol=0, atol=1e-14)


def test_patch_divergence_p1():
    """P1-P1: B I(v) = -M_p (div v) 1 for linear v (constant divergence)."""
    N = 3
    lev = fe.Level(N, 1)
    c = lev.vpos()
    v = [lambda x, y, z: 2 * x + y, lambda x, y, z: -y + z, lambda x, y, z: 3 * z - x]
    Bv = sum(lev.B[d] @ _poly_vals(c, v[d]) for d in range(3))
    assert np.allclose(Bv, -4.0 * (lev.Mp @ np.ones(lev.np_)), rtol=0, atol=1e-14)


def test_local_p2_stiffness_reference_values():
    """Reference tetrahedron (0, e1, e2, e3): the P2 stiffness (degree-2
    integrand) equals the 4-point degree-2 exact quadrature of the hand-written
    basis gradients; P2 basis integrals are -|T|/20 (vertex), |T|/5 (edge)."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    K = fe.local_stiffness(X, 2)
    assert np.allclose(K.sum(axis=1), 0.0, atol=1e-15)
    # degree-2 exact 4-point rule on the reference tetrahedron
    a, b = 0.5854101966249685, 0.1381966011250105
    pts = np.array([[b, b, b], [a, b, b], [b, a, b], [b, b, a]])
    w = np.full(4, 1.0 / 24.0)

    def grads(p):
        lam = np.array([1 - p.sum(), p[0], p[1], p[2]])
        g = np.array([[-1, -1, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
        out = [(4 * lam[i] - 1) * g[i] for i in range(4)]
        out += [4 * (lam[j] * g[i] + lam[i] * g[j]) for (i, j) in mesh.P2_EDGES]
        return np.array(out)
    Kq = sum(wi * grads(p) @ grads(p).T for wi, p in zip(w, pts))
    assert np.allclose(K, Kq, rtol=0, atol=1e-14)
    M = fe.local_mass(X, 2)
    load = M.sum(axis=1)
    # vertex basis integrate to -|T|/20, edge basis to |T|/5
    vol = 1.0 / 6.0
    assert np.allclose(load[:4], -vol / 20.0, atol=1e-16)
    assert np.allclose(load[4:], vol / 5.0, atol=1e-16)


# ------------------------------------------------------ variable viscosity
# Reading of the paper's operator with a viscosity field (not in the paper's
# experiments): a_ij = sum_T nu_T int_T grad phi_i . grad phi_j per velocity
# component, nu_T the mean of the four vertex values of nu.  For a linear nu
# that mean is the exact element mean, which gives closed forms.
def _nu_linear(x, y, z):
    return 1.0 + 2.0 * x + 3.0 * y + 5.0 * z          # grad nu = (2, 3, 5), int_cube nu = 6


def _nu_level(N, vorder, fn):
    cp = mesh.p1_coords(N) / float(N)
    return fe.Level(N, vorder, fn(cp[:, 0], cp[:, 1], cp[:, 2]))


def test_variable_viscosity_p1_rows_linear_nu():
    """P1, linear nu, linear q: int nu grad phi_i . grad q = -(grad nu . grad q)
    int phi_i on interior rows (integration by parts, no boundary term), and
    int phi_i is the lumped mass."""
    N = 4
    lev = _nu_level(N, 1, _nu_linear)
    c = lev.vpos()
    q = lambda x, y, z: 2 * x - y + 3 * z + 0.25              # grad nu . grad q = 4 - 3 + 15 = 16
    got = (lev.A @ _poly_vals(c, q))[lev.vint]
    want = -16.0 * lev.ML[lev.vint]
    assert np.allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("vorder", [1, 2])
def test_variable_viscosity_bilinear_form_linear_nu(vorder):
    """I(r)^T A(nu) I(q) = (grad r . grad q) int_cube nu for linear r, q (both
    in the element space) and linear nu: 6 * (2 - 2 - 1) = -6."""
    N = 3
    lev = _nu_level(N, vorder, _nu_linear)
    c = lev.vpos()
    r = lambda x, y, z: x - 2 * y + z
    q = lambda x, y, z: 2 * x + y - z + 1.0                    # grad r . grad q = 2 - 2 - 1 = -1
    val = _poly_vals(c, r) @ (lev.A @ _poly_vals(c, q))
    assert abs(val - (-6.0)) < 1e-12


def test_variable_viscosity_p2_vertex_rows_vanish():
    """P2, any element-wise constant nu, linear q: the integral of the gradient
    of a quadratic vertex basis function over each element is zero
    (int (4 lam - 1) = 0), so A(nu) I(q) vanishes on the vertex rows; the
    edge rows do not (they carry nu_T |T| grad q . (grad lam_a + grad lam_b))."""
    N = 4
    g = np.random.default_rng(5)
    nu_nodes = np.exp(g.standard_normal((N + 1) ** 3))
    lev = fe.Level(N, 2, nu_nodes)
    c = lev.vpos()
    q = lambda x, y, z: 3 * x - 2 * y + 0.5 * z
    Aq = lev.A @ _poly_vals(c, q)
    vert = np.all(lev.vcoords % 2 == 0, axis=1) & lev.vint
    edge = ~np.all(lev.vcoords % 2 == 0, axis=1) & lev.vint
    assert np.abs(Aq[vert]).max() < 1e-13
    assert np.abs(Aq[edge]).max() > 1e-3


@pytest.mark.parametrize("vorder", [1, 2])
def test_variable_viscosity_scaling_symmetry_row_sums(vorder):
    """A(c 1) = c A(1); A(nu) symmetric with zero row sums for a random
    positive nu; A(nu) with nu = 1 equals the constant-coefficient matrix."""
    N = 3
    n1 = (N + 1) ** 3
    A1 = fe.Level(N, vorder).A
    Ac = fe.Level(N, vorder, np.full(n1, 3.7)).A
    assert abs(Ac - 3.7 * A1).max() < 1e-13 * abs(Ac).max()
    assert abs(fe.Level(N, vorder, np.ones(n1)).A - A1).max() < 1e-15 * abs(A1).max()
    nu = np.exp(np.random.default_rng(7).standard_normal(n1))
    A = fe.Level(N, vorder, nu).A
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-12 * abs(A).max()
