"""The oracle against the coupled convergence test of Sec. 5.1 (tab:convergence).

Reading of the set-up: "L = 0.1 m on each side, centred about the origin"
is taken as the half-width, i.e. the periodic cube spans [-0.1, 0.1] m (the
cosines of eq:convergeE/H then hold two periods).  With that reading the
oracle's H error levels agree with the table to ~1 % and the E levels to
~11 %; with a 0.1 m cube they come out 4x (H) and 14x (E) below it.  The M
error levels depend on the material averaging stencils, which the paper
does not give, so they are reported but only their rates are pinned.

The default test compares the first error column (32^3 vs 64^3, ~10 s); the
full table with rates needs a 128^3 run (~4 min) and runs when
MM_SLOW_TESTS=1.
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
