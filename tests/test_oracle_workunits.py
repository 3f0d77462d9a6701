"""Pins of the work-unit model against the values printed in Sec. 4 and
Tab. fmg-table (fixtures in tests/golden/)."""
import os
from fractions import Fraction

import pytest

from oracle import mesh, workunits as wu
from oracle.multigrid import Params

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    for line in open(os.path.join(GOLD, name)):
        if line.strip() and not line.startswith("#"):
            yield line.split()


@pytest.mark.parametrize("row", list(_rows("fmg_table.txt")))
def test_fmg_work_units_match_paper(row):
    disc, npre, npost, ninc, kap, gs, xi, W = row
    prm = Params(int(npre), int(npost), int(ninc), int(kap), gs, int(xi))
    got = wu.fmg_bound(prm, 1 if disc == "P1P1" else 2)
    digits = len(W.split(".")[1])
    assert round(got, digits) == float(W)


def _limit_ratio(f, level=60):
    return f(level)


def test_asymptotic_ratios():
    gold = {r[0]: Fraction(int(r[1]), int(r[2])) for r in _rows("wu_ratios.txt")}
    nt = mesh.n_tet
    L = 40
    n = 2 ** L
    unk_p2 = 3 * (nt(n - 3) + 6 * nt(n - 2) + nt(n - 1)) + nt(n - 3)
    unk_p1 = 4 * nt(2 * n - 3)
    assert abs(unk_p2 / unk_p1 - float(gold["unknowns_p2p1_over_p1p1_next_level"])) < 1e-9
    A2, B2, C2 = wu.block_costs(2, L)
    A1, B1, C1 = wu.block_costs(1, L + 1)
    assert abs(A2 / A1 - float(gold["A_p2p1_over_A_p1p1_next_level"])) < 1e-9
    assert abs(B2 / B1 - float(gold["B_p2p1_over_B_p1p1_next_level"])) < 1e-9
    assert abs((A2 + 2 * B2 + C2) / (A1 + 2 * B1 + C1) - float(gold["op_p2p1_over_op_p1p1_next_level"])) < 1e-9
    a2, b2, c2 = wu.normalised_blocks(2)
    a1, b1, c1 = wu.normalised_blocks(1)
    assert abs(a2 - float(gold["A_share_p2p1"])) < 1e-9
    assert abs(b2 - float(gold["B_share_p2p1"])) < 1e-9
    assert abs(a1 - float(gold["A_share_p1p1"])) < 1e-9
    assert abs(c1 - float(gold["C_share_p1p1"])) < 1e-9
    assert abs(wu.uzawa_cost(2, "f", 1) - float(gold["uzawa_p2p1_Af_xi1"])) < 1e-9
    assert abs(wu.uzawa_cost(2, "s", 1) - float(gold["uzawa_p2p1_As_xi1"])) < 1e-9


def test_level_sum_below_bound():
    """The level-by-level sum is bounded by the geometric-series estimate."""
    for vo in (1, 2):
        prm = Params(1, 2, 1, 1, "f", 3)
        assert wu.fmg_exact_sum(prm, vo, 0, 7) <= wu.fmg_bound(prm, vo) + 1e-9
