"""Parameter study of the FMG solver (paper Sec. 5.1, search space S).

Host-side driver around the C ABI: for every tuple s = (nu_pre, nu_post,
nu_inc, kappa, A_hat, xi) of the search space it runs one FMG solve on the
GPU (Alg. fmg), evaluates the errors of eq. error on the next finer level and
their ratios gamma_u, gamma_p to the discretisation error (eq. gamma, the
discrete solution being an FMG solve continued with V-cycles to
||r|| <= 1e-12 ||b||), and records the work units of the Sec. 4 model that
the library reports.  From the table it selects, as Tab. fmg-table does, the
tuple of least work under upper bounds (gamma_u_hat, gamma_p_hat) with kappa =
1, and the least error reachable within a given work (the data of the
paper's min-error-for-work figure).  All arithmetic runs in the library.
"""
import itertools
import time

import numpy as np

from . import hhg

# (A_hat, xi) pairs of the search space: forward Gauss-Seidel with 1..4
# sweeps, symmetric with 1..2
SMOOTHERS = [(hhg.HHG_GS_FWD, 1), (hhg.HHG_GS_FWD, 2), (hhg.HHG_GS_FWD, 3), (hhg.HHG_GS_FWD, 4),
             (hhg.HHG_GS_SYM, 1), (hhg.HHG_GS_SYM, 2)]
BOUNDS = [(1.1, 2.0), (1.1, 5.0), (2.0, 10.0), (2.0, 2.0)]


def search_space():
    """The 768 tuples: 0 <= nu_pre, nu_post, nu_inc <= 3, kappa in {1, 2},
    (A_hat, xi) from SMOOTHERS."""
    out = []
    for pre, post, inc, kappa in itertools.product(range(4), range(4), range(4), (1, 2)):
        for gs, xi in SMOOTHERS:
            out.append((pre, post, inc, kappa, gs, xi))
    return out


def tuple_name(s):
    return f"({s[0]},{s[1]},{s[2]},{s[3]},{'A_f' if s[4] == hhg.HHG_GS_FWD else 'A_s'},{s[5]})"


class GammaEvaluator:
    """Errors of eq. error for one problem on a hierarchy: the computed
    finest-level solution is prolonged to level L+1 (a second hierarchy
    holding levels L, L+1), the exact solution's nodal values there are
    subtracted, both pressures are taken to zero mean, and the velocity and
    pressure parts are measured in the consistent-mass norm."""

    def __init__(self, torch, P, prob):
        self.torch = torch
        self.P = P
        L = P.lmax
        self.L = L
        mesh = hhg.hhg_mesh_cube(P.ctx, P.mr)
        try:
            self.ev = hhg.hhg_hier_create(mesh, P.disc, L, L + 1)
        finally:
            hhg.hhg_mesh_destroy(mesh)
        _, _, vw, _ = hhg.hhg_vec_layout(self.ev, L + 1)
        lat = P.lattice(L + 1, prob.u, prob.p)
        src = torch.from_numpy(np.ascontiguousarray(lat)).to(P.dev)
        self.xs = torch.zeros(vw, dtype=torch.float64, device=P.dev)
        hhg.hhg_vec_from_lattice(self.ev, L + 1, src, self.xs)
        self.e = torch.empty_like(self.xs)
        self.me = torch.empty_like(self.xs)

    def errors(self, xL):
        self.e.zero_()
        hhg.hhg_prolong_add(self.ev, self.L, xL, self.e)
        self.e -= self.xs
        hhg.hhg_project_mean_zero(self.ev, self.L + 1, self.e)
        hhg.hhg_apply(self.ev, self.L + 1, hhg.HHG_OP_MASS, self.e, self.me)
        du, dp = hhg.hhg_dots(self.ev, self.L + 1, self.e, self.me)
        return float(np.sqrt(du)), float(np.sqrt(dp))

    def close(self):
        if self.ev is not None:
            self.torch.cuda.synchronize()
            hhg.hhg_hier_destroy(self.ev)
            self.ev = None


def discrete_solution(P, bs, x0, omega_inv, rtol=1e-12):
    """FMG continued with V(3,3) cycles until ||r|| <= rtol ||b|| (the
    discrete solution of eq. gamma)."""
    xi = 1 if P.disc == hhg.HHG_P1P1 else 3
    xd = x0.clone()
    st = hhg.hhg_fmg_solve(P.h, xd, bs, hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_FWD, xi, omega_inv, rtol=rtol,
                                                           max_cycles=300))
    return xd, st


def run(torch, P, prob, omega_inv, tuples, log=None, every=64):
    """FMG solve, errors and gamma for every tuple; returns the rows and the
    discretisation errors."""
    bs = P.rhs(prob)
    x0 = P.boundary(prob)
    gev = GammaEvaluator(torch, P, prob)
    try:
        xd, st = discrete_solution(P, bs, x0, omega_inv)
        ed = gev.errors(xd)
        if log:
            log(f"[sweep] discrete solution: {st.cycles} cycles, rel res {st.rel_res:.1e}, "
                f"errors u {ed[0]:.4e} p {ed[1]:.4e}")
        x = torch.empty_like(x0)
        rows = []
        t0 = time.perf_counter()
        for q, s in enumerate(tuples):
            x.copy_(x0)
            prm = hhg.solver_params(*s, omega_inv)
            st = hhg.hhg_fmg_solve(P.h, x, bs, prm)
            eu, ep = gev.errors(x)
            rows.append({"s": list(s), "name": tuple_name(s), "wu": st.work_units, "gamma_u": eu / ed[0],
                         "gamma_p": ep / ed[1], "err_u": eu, "err_p": ep, "seconds": st.seconds})
            if log and (q + 1) % every == 0:
                log(f"[sweep] {q + 1}/{len(tuples)} tuples, {time.perf_counter() - t0:.1f} s")
        return rows, ed
    finally:
        gev.close()


def best_under_bounds(rows, bounds=BOUNDS, kappa=1):
    """Tab. fmg-table: for each (gamma_u_hat, gamma_p_hat), the tuple with
    kappa = `kappa` and least work whose gammas are within the bounds (ties:
    smaller gamma_p), and the one of least measured solve time."""
    out = []
    for gu, gp in bounds:
        ok = [r for r in rows if r["s"][3] == kappa and r["gamma_u"] <= gu and r["gamma_p"] <= gp]
        best = min(ok, key=lambda r: (round(r["wu"], 9), r["gamma_p"])) if ok else None
        fastest = min(ok, key=lambda r: r["seconds"]) if ok else None
        out.append({"bounds": [gu, gp], "best": best, "fastest": fastest})
    return out


def min_error_for_work(rows, key):
    """For each work value reached by some tuple, the least gamma (key =
    'gamma_u' or 'gamma_p') among tuples of at most that work: the lower
    envelope plotted against work."""
    pts = sorted((r["wu"], r[key], r["name"]) for r in rows)
    env, best = [], float("inf")
    for wu, g, name in pts:
        if g < best:
            best = g
            env.append({"wu": wu, key: g, "name": name})
    return env
