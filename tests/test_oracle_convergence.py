"""The oracle against the coupled convergence test of Sec. 5.1 (tab:convergence).

Reading of the set-up: the paper gives the cube's size as 0.1 m per side,
centred on the origin; we take 0.1 m as the half-width, so the periodic cube
spans [-0.1, 0.1] m and the cosines of eq:convergeE/H hold two periods.
With that reading the oracle's H error levels agree with the table to ~1 %
and the E levels to ~11 %; with a 0.1 m cube they come out 4x (H) and 14x
(E) below it.  The M error levels depend on the material averaging
stencils, which the paper does not give, so they are reported but only
their rates are pinned.

Default tests: the first error column (32^3 vs 64^3, ~10 s), and the rates
of all 15 variables on a 16^3 / 32^3 / 64^3 ladder over a shorter common
time (2, 4, 8 steps; ~10 s), which must be second order as the table's are.
The paper's own ladder, 32^3 / 64^3 / 128^3 over 5, 10, 20 steps, needs a
128^3 run (~4 min) and runs when MM_SLOW_TESTS=1.
"""
import json
import math
import os

import pytest

from tests import convergence_case as CC

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "convergence_table.json")))
SIDE = 0.2


def _errors(N1, N2, cache={}):
    for N in (N1, N2):
        if N not in cache:
            cache[N] = CC.run(N, side=SIDE)
    return CC.l1_error(cache[N1], cache[N2])


def test_rates_are_second_order_on_a_short_ladder():
    """16^3, 32^3, 64^3 run to the same physical time (2, 4, 8 steps at CFL
    0.9): every E, H and M component converges at rate 2 (measured
    1.98-2.02)."""
    runs = [CC.run(N, side=SIDE, steps=N // 8) for N in (16, 32, 64)]
    e1 = CC.l1_error(runs[0], runs[1])
    e2 = CC.l1_error(runs[1], runs[2])
    assert len(e1) == 15
    for nm in e1:
        rate = math.log2(e1[nm] / e2[nm])
        assert 1.95 < rate < 2.05, (nm, rate)


def test_first_error_column_matches_table():
    e = _errors(32, 64)
    rows = GOLD["rows"]
    for nm in ("Ex", "Ey", "Ez"):
        assert abs(e[nm] / rows[nm][0] - 1) < 0.15, (nm, e[nm], rows[nm][0])
    for nm in ("Hx", "Hy", "Hz"):
        assert abs(e[nm] / rows[nm][0] - 1) < 0.03, (nm, e[nm], rows[nm][0])
    # M levels: same order of magnitude as the table (stencils unpinned)
    for f in "xyz":
        for c in "xyz":
            assert 0.1 < e["M" + f + c] / rows["M" + c][0] < 10


@pytest.mark.skipif(os.environ.get("MM_SLOW_TESTS") != "1", reason="128^3 run takes ~4 min; set MM_SLOW_TESTS=1")
def test_full_table_rates_are_second_order():
    e1 = _errors(32, 64)
    e2 = _errors(64, 128)
    rows = GOLD["rows"]
    for nm in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"):
        assert abs(e2[nm] / rows[nm][1] - 1) < (0.15 if nm[0] == "E" else 0.03), (nm, e2[nm])
    for nm in e1:
        rate = math.log2(e1[nm] / e2[nm])
        assert 1.95 < rate < 2.05, (nm, rate)
