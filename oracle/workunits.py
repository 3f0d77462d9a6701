"""Work-unit cost model (oracle; test infrastructure).

Paper Sec. 4.  A stencil with n entries costs 2n operations; velocity blocks
count three components.  Block costs per level from eq. cost-block-p2p1-b,
cost-block-p2p1-a, cost-block-p2p1-c, cost-block-p1p1-ab, cost-block-p1p1-c
with the interior unknown counts of Tab. unknown-count and the stencil sizes
of Tab. stencil-count.  W(calA) = W(A) + W(B^T) + W(B) + W(C) with
W(B^T) ~ W(B); one forward Gauss-Seidel sweep costs W(A), a symmetric one
2 W(A); W(P^{-1}) = W(A_hat^{-1}) + W(B^T) + W(B) + W(C) with xi sweeps in
A_hat^{-1}.  Variable V-cycle bound eq. bound-var-v-cycle and FMG bound eq.
cost-var-fmg; results are normalised by W(calA_L) (eq. work-unit).
"""
from .mesh import n_tet


def block_costs(vorder, level):
    """(W(A), W(B), W(C)) on one macro-cell of the given refinement level."""
    n = 2 ** level
    if vorder == 2:
        WA = 3 * ((2 * 65) * n_tet(n - 3) + (2 * 146) * n_tet(n - 2) + (2 * 19) * n_tet(n - 1))
        WB = 3 * (2 * 65) * n_tet(n - 3)
        WC = 0
    else:
        WA = 3 * (2 * 15) * n_tet(n - 3)
        WB = WA
        WC = (2 * 15) * n_tet(n - 3)
    return WA, WB, WC


def normalised_blocks(vorder, level=40):
    """Block costs divided by W(calA) (large level = the asymptotic limit)."""
    WA, WB, WC = block_costs(vorder, level)
    Wop = WA + 2 * WB + WC
    return WA / Wop, WB / Wop, WC / Wop


def uzawa_cost(vorder, gs, xi, level=40):
    """W(P^{-1}) in WU: xi sweeps of A_f (or A_s = 2 sweeps) + B^T + B + C."""
    a, b, c = normalised_blocks(vorder, level)
    sweeps = xi * (2 if gs == "s" else 1)
    return sweeps * a + 2 * b + c


def vcycle_bound(prm, vorder, level=40):
    """W*(V^L) = 8/7 W(V_L^L) + 16/49 nu_inc W(P_L^{-1})  (eq. bound-var-v-cycle)."""
    wp = uzawa_cost(vorder, prm.gs, prm.xi, level)
    wvll = (prm.nu_pre + prm.nu_post) * wp + 1.0
    return 8.0 / 7.0 * wvll + 16.0 / 49.0 * prm.nu_inc * wp


def fmg_bound(prm, vorder, level=40):
    """W(FMG^L) <~ 8 kappa / 7 W*(V^L)  (eq. cost-var-fmg), in WU."""
    return 8.0 * prm.kappa / 7.0 * vcycle_bound(prm, vorder, level)


def fmg_exact_sum(prm, vorder, Lmin, Lmax):
    """Level-by-level sum of the same model, sum_l kappa W(V^l) / W(calA_L),
    using the exact interior counts of every level (no geometric series)."""
    WA_L, WB_L, WC_L = block_costs(vorder, Lmax)
    Wop_L = WA_L + 2 * WB_L + WC_L
    tot = 0.0
    for lf in range(Lmin + 1, Lmax + 1):
        for l in range(Lmin + 1, lf + 1):
            WA, WB, WC = block_costs(vorder, l)
            sweeps = prm.xi * (2 if prm.gs == "s" else 1)
            wp = sweeps * WA + 2 * WB + WC
            wop = WA + 2 * WB + WC
            its = prm.nu_pre + prm.nu_post + 2 * (lf - l) * prm.nu_inc
            tot += prm.kappa * (its * wp + wop)
    return tot / Wop_L
