"""Seeded synthetic inputs: manufactured solutions, forcing and viscosity
fields, and macro meshes T_0 (vertex coordinates and tetrahedra).

Problem data only -- analytic fields evaluated at given coordinates and seeded
random draws.  It contains none of the solver's arithmetic; both the library's
tests/benchmark and the CPU oracle take their inputs from here.

Seeds: base 13513; workload k uses 13513 + 1000 k.  Host RNG is
numpy.random.Generator(PCG64(seed)).
"""
from dataclasses import dataclass

import numpy as np

SEED_BASE = 13513
PI = np.pi


@dataclass
class Fields:
    """u(x,y,z) -> (3, n), p(x,y,z) -> (n,), f(x,y,z) -> (3, n)."""
    u: object
    p: object
    f: object
    name: str = ""


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _z(x):
    return np.zeros_like(np.asarray(x, dtype=float))


def paper_cube():
    """Analytic solution of the paper's cube benchmark (Sec. 5.1.1):
    u = (-4 cos 4z, 8 cos 8x, -2 cos 2y), p = sin 4x sin 8y sin 2z, f = -lap u + grad p."""
    def u(x, y, z):
        return np.stack([-4 * np.cos(4 * z), 8 * np.cos(8 * x), -2 * np.cos(2 * y)])

    def p(x, y, z):
        return np.sin(4 * x) * np.sin(8 * y) * np.sin(2 * z)

    def f(x, y, z):
        return np.stack([
            -64 * np.cos(4 * z) + 4 * np.cos(4 * x) * np.sin(8 * y) * np.sin(2 * z),
            512 * np.cos(8 * x) + 8 * np.sin(4 * x) * np.cos(8 * y) * np.sin(2 * z),
            -8 * np.cos(2 * y) + 2 * np.sin(4 * x) * np.sin(8 * y) * np.cos(2 * z)])
    return Fields(u, p, f, "paper_cube")


def sine_cube():
    """Smooth divergence-free field with zero net boundary flux:
    u = (s, s, sin(pi(x+y)) cos(pi z)), s = sin(pi x) sin(pi y) sin(pi z),
    p = cos(pi x) cos(pi y) cos(pi z) (zero mean); f = 3 pi^2 u + grad p."""
    def u(x, y, z):
        s = np.sin(PI * x) * np.sin(PI * y) * np.sin(PI * z)
        return np.stack([s, s, np.sin(PI * (x + y)) * np.cos(PI * z)])

    def p(x, y, z):
        return np.cos(PI * x) * np.cos(PI * y) * np.cos(PI * z)

    def f(x, y, z):
        uu = u(x, y, z)
        gp = np.stack([-PI * np.sin(PI * x) * np.cos(PI * y) * np.cos(PI * z),
                       -PI * np.cos(PI * x) * np.sin(PI * y) * np.cos(PI * z),
                       -PI * np.cos(PI * x) * np.cos(PI * y) * np.sin(PI * z)])
        return 3 * PI ** 2 * uu + gp
    return Fields(u, p, f, "sine_cube")


def quadratic_exact():
    """u = (y^2, z^2, x^2), p = x + y + z - 3/2, f = (-1, -1, -1): inside the
    Taylor-Hood space, so the discrete solution reproduces it."""
    def u(x, y, z):
        return np.stack([y * y, z * z, x * x])

    def p(x, y, z):
        return x + y + z - 1.5

    def f(x, y, z):
        return np.stack([-np.ones_like(x)] * 3)
    return Fields(u, p, f, "quadratic_exact")


def linear_exact():
    """u = (y, z, x), p = 0, f = 0: reproduced by the P1-P1 discretisation."""
    def u(x, y, z):
        return np.stack([y, z, x])

    def p(x, y, z):
        return _z(x)

    def f(x, y, z):
        return np.stack([_z(x)] * 3)
    return Fields(u, p, f, "linear_exact")


# Outflow (natural Neumann) boundary on the face x = 1 (Sec. 2: du/dn = n p on
# the Neumann part), Dirichlet on the other five faces.
OUTFLOW_FACES = (1,)


def outflow_cube():
    """Smooth solution satisfying the outflow condition on x = 1:
    u = (a q, a' chi_y, a' chi_z), p = a' q with a = x^3 - 3 x^2,
    chi = sin(pi y) sin(pi z), q = 2 pi^2 chi (= -lap_yz chi), so div u = 0,
    du/dx = (a' q, a'' chi_y, a'' chi_z) = (p, 0, 0) at x = 1 (a''(1) = 0);
    f = -lap u + grad p = (2 pi^2 a q, (4 pi^2 a' - 6) chi_y, (4 pi^2 a' - 6) chi_z)."""
    def parts(x, y, z):
        a = x ** 3 - 3 * x ** 2
        da = 3 * x ** 2 - 6 * x
        sy, cy, sz, cz = np.sin(PI * y), np.cos(PI * y), np.sin(PI * z), np.cos(PI * z)
        chi = sy * sz
        return a, da, chi, PI * cy * sz, PI * sy * cz

    def u(x, y, z):
        a, da, chi, chy, chz = parts(x, y, z)
        return np.stack([a * 2 * PI ** 2 * chi, da * chy, da * chz])

    def p(x, y, z):
        a, da, chi, _, _ = parts(x, y, z)
        return da * 2 * PI ** 2 * chi

    def f(x, y, z):
        a, da, chi, chy, chz = parts(x, y, z)
        g = 4 * PI ** 2 * da - 6.0
        return np.stack([2 * PI ** 2 * a * 2 * PI ** 2 * chi, g * chy, g * chz])
    return Fields(u, p, f, "outflow_cube")


def outflow_polynomial(vorder):
    """Fields inside the element spaces that satisfy the outflow condition on
    x = 1, so the discrete solution reproduces them: P2-P1 u = (y^2 - z^2,
    x^2 - 2 x, 3), p = 1 - x, f = (-1, -2, 0); P1-P1 u = (x, -y, 0), p = 1,
    f = 0."""
    if vorder == 2:
        def u(x, y, z):
            return np.stack([y * y - z * z, x * x - 2 * x, 3.0 + _z(x)])

        def p(x, y, z):
            return 1.0 - x

        def f(x, y, z):
            return np.stack([-1.0 + _z(x), -2.0 + _z(x), _z(x)])
    else:
        def u(x, y, z):
            return np.stack([np.asarray(x, float) + _z(x), -np.asarray(y, float) + _z(x), _z(x)])

        def p(x, y, z):
            return 1.0 + _z(x)

        def f(x, y, z):
            return np.stack([_z(x)] * 3)
    return Fields(u, p, f, f"outflow_polynomial_p{vorder}")


def fourier_forcing(seed, modes=8, kmax=4):
    """f = sum_m a_m sin(2 pi k_m . x + phi_m); k_m uniform in {-kmax..kmax}^3 \\ 0,
    a_m ~ N(0,1)^3 / |k_m|^2, phi_m ~ U[0, 2 pi); u = 0 on the boundary, p unknown."""
    g = rng(seed)
    ks, amps, phis = [], [], []
    while len(ks) < modes:
        k = g.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    for k in ks:
        amps.append(g.standard_normal(3) / float(k @ k))
        phis.append(g.uniform(0.0, 2 * PI))

    def f(x, y, z):
        out = np.zeros((3,) + np.shape(x))
        for k, a, ph in zip(ks, amps, phis):
            s = np.sin(2 * PI * (k[0] * x + k[1] * y + k[2] * z) + ph)
            out += a.reshape((3,) + (1,) * np.ndim(s)) * s
        return out

    def u(x, y, z):
        return np.stack([_z(x)] * 3)

    def p(x, y, z):
        return _z(x)
    return Fields(u, p, f, f"fourier_{seed}")


def gaussian_bump_viscosity(seed, bumps=8, width=0.15, ratio=100.0, N_ref=None):
    """nu = exp(ln(ratio) (G - min G)/(max G - min G)), G = sum_b a_b exp(-|x-c_b|^2/(2 w^2)),
    a_b ~ N(0,1), c_b ~ U[0,1]^3; min/max over the nodes of the lattice N_ref."""
    g = rng(seed)
    a = g.standard_normal(bumps)
    c = g.uniform(0.0, 1.0, size=(bumps, 3))

    def G(x, y, z):
        out = np.zeros(np.shape(x))
        for ab, cb in zip(a, c):
            out += ab * np.exp(-((x - cb[0]) ** 2 + (y - cb[1]) ** 2 + (z - cb[2]) ** 2) / (2 * width ** 2))
        return out

    n = 32 if N_ref is None else N_ref
    t = np.linspace(0.0, 1.0, n + 1)
    X, Y, Z = np.meshgrid(t, t, t, indexing="ij")
    GG = G(X, Y, Z)
    gmin, gmax = float(GG.min()), float(GG.max())

    def nu(x, y, z):
        return np.exp(np.log(ratio) * (G(x, y, z) - gmin) / (gmax - gmin))
    return nu


def lognormal_viscosity(seed, modes=8, kmax=2, ratio=100.0):
    """nu = exp(sigma G), G a unit-variance sum of `modes` Fourier modes,
    sigma = ln(ratio) / 4."""
    g = rng(seed)
    ks, phis = [], []
    while len(ks) < modes:
        k = g.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    amp = g.standard_normal(modes)
    for _ in ks:
        phis.append(g.uniform(0.0, 2 * PI))
    scale = np.sqrt(2.0 / np.sum(amp ** 2))
    sigma = np.log(ratio) / 4.0

    def nu(x, y, z):
        G = np.zeros(np.shape(x))
        for k, a, ph in zip(ks, amp, phis):
            G += a * np.sin(2 * PI * (k[0] * x + k[1] * y + k[2] * z) + ph)
        return np.exp(sigma * scale * G)
    return nu


def normal_vector(seed, n):
    """Seeded N(0,1) float64 vector."""
    return rng(seed).standard_normal(n)


# ------------------------------------------------------------ macro meshes
# Input geometry only: (xyz (nv, 3) float64, tets (nt, 4) int64).

def cube24():
    """The unit cube as 24 tetrahedra: each face split into 4 triangles at its
    centre, each triangle joined to the cube's centre (15 vertices, 50 edges,
    60 faces).  Uniform refinement gives 4.29e6 P1-P1 unknowns at L = 6 and
    3.36e6 P2-P1 unknowns at L = 5, the counts quoted for the cube benchmark
    of Sec. 5.1.1."""
    xyz = [(i, j, k) for k in (0, 1) for j in (0, 1) for i in (0, 1)]          # corners 0..7
    cid = {c: n for n, c in enumerate(xyz)}
    faces = []
    for d in range(3):
        for side in (0, 1):
            cen = [0.5, 0.5, 0.5]
            cen[d] = side
            xyz.append(tuple(cen))
            a, b = [e for e in range(3) if e != d]
            ring = []
            for (s, t) in ((0, 0), (1, 0), (1, 1), (0, 1)):     # around the face
                c = [0, 0, 0]
                c[d], c[a], c[b] = side, s, t
                ring.append(cid[tuple(c)])
            faces.append((len(xyz) - 1, ring))
    xyz.append((0.5, 0.5, 0.5))
    body = len(xyz) - 1
    tets = []
    for fc, ring in faces:
        for q in range(4):
            tets.append((body, fc, ring[q], ring[(q + 1) % 4]))
    return np.array(xyz, dtype=float), np.array(tets, dtype=np.int64)


_KUHN_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def kuhn_cube(N):
    """The unit cube as N^3 sub-cubes of 6 Kuhn tetrahedra each (vertices of
    a tetrahedron along the path 0, e_a, e_a + e_b, (1,1,1))."""
    n1 = N + 1
    xyz = np.array([(i, j, k) for k in range(n1) for j in range(n1) for i in range(n1)], float) / N
    idx = lambda c: c[0] + n1 * (c[1] + n1 * c[2])
    tets = []
    for k in range(N):
        for j in range(N):
            for i in range(N):
                for p in _KUHN_PERMS:
                    c = [i, j, k]
                    t = [idx(c)]
                    for a in p:
                        c[a] += 1
                        t.append(idx(c))
                    tets.append(t)
    return xyz, np.array(tets, dtype=np.int64)


def jittered_cube(seed, N=2, amp=0.12):
    """kuhn_cube(N) with every vertex moved by a seeded uniform offset of up
    to amp / N per coordinate, except along the normals of the cube faces it
    lies on (the domain stays the unit cube, the mesh is no Kuhn partition)."""
    xyz, tets = kuhn_cube(N)
    off = rng(seed).uniform(-amp / N, amp / N, size=xyz.shape)
    on_face = (np.abs(xyz) < 1e-12) | (np.abs(xyz - 1.0) < 1e-12)
    return xyz + np.where(on_face, 0.0, off), tets


def box_cube24(nx, ny, nz):
    """An nx x ny x nz box of unit cubes, each split as in cube24 (shared
    vertices merged)."""
    xyz0, tets0 = cube24()
    pts, tets = {}, []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                ids = []
                for v in xyz0 + np.array([i, j, k], float):
                    key = tuple(np.round(v * 2).astype(int))
                    ids.append(pts.setdefault(key, len(pts)))
                tets += [[ids[a] for a in t] for t in tets0]
    xyz = np.zeros((len(pts), 3))
    for key, q in pts.items():
        xyz[q] = np.array(key, float) / 2
    return xyz, np.array(tets, dtype=np.int64)


def boundary_faces_on_planes(xyz, tets, faces):
    """Boundary triangles (sorted vertex triples) of the mesh that lie on the
    listed faces of the unit cube (0: x = 0, 1: x = 1, 2: y = 0, 3: y = 1,
    4: z = 0, 5: z = 1)."""
    count = {}
    for t in tets:
        for drop in range(4):
            f = tuple(sorted(int(v) for q, v in enumerate(t) if q != drop))
            count[f] = count.get(f, 0) + 1
    out = []
    for f, c in sorted(count.items()):
        if c != 1:
            continue
        P = np.asarray(xyz)[list(f)]
        for face in faces:
            d, val = face // 2, float(face % 2)
            if np.all(np.abs(P[:, d] - val) < 1e-12):
                out.append(f)
                break
    return out
