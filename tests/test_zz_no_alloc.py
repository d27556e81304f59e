"""mm_step_noalloc, the stepping entry point for callers that cannot allocate,
against mm_step through the C ABI.

Both entry points run the same kernels; the variant takes the sub-step
control (final-count words, barrier state, residual partials) from the
library's fixed per-device array instead of the context.  The bar is the
FP64 parity bar of the HIP path, bit for bit: every field (E, H and the nine
M components), every probe series and integral, every iteration count.

Two contexts in a row, the second on a smaller grid with fewer residual
partials, so the second call runs on whatever the first left in the array;
each also switches between the two entry points within one run.  A random
start makes the sub-steps take several iterations.
"""
import numpy as np
import pytest

import workloads as W
from tests import parity_util as PU

pytestmark = pytest.mark.gpu
FIELDS = PU.E_H + PU.M_NAMES


def _noalloc(sim, n):
    return sim._lib.mm_step_noalloc(sim._ctx, int(n))


def _assert_same(ref, sim, nprobes):
    for nm in FIELDS:
        a, b = sim.field(nm), ref.field(nm)
        assert np.array_equal(a, b), (nm, float(np.max(np.abs(a - b))))
    assert list(sim.stats()) == list(ref.stats())
    for pid in range(nprobes):
        s1, S1 = sim.probe(pid)
        s0, S0 = ref.probe(pid)
        assert np.array_equal(s1, s0) and S1 == S0, pid


def _run(cfg, precision, warm, n1, n2):
    import paper_2103_12819_amd as mm
    print(f"no-alloc case {cfg.name} {cfg.n} {precision}: {warm} + {n1} + 1 + {n2} steps", flush=True)
    ref = mm.from_config(cfg, precision=precision)
    ref.step(warm + n1 + 1 + n2)
    sim = mm.from_config(cfg, precision=precision)
    sim.step(warm)                      # makes the iteration log and probe storage
    assert _noalloc(sim, n1) == 0, sim._lib.mm_last_error(sim._ctx)
    sim.step(1)                         # back to the context's own control words
    assert _noalloc(sim, n2) == 0, sim._lib.mm_last_error(sim._ctx)
    _assert_same(ref, sim, len(cfg.probes))
    it = sim.stats()
    ref.close()
    sim.close()
    return it


def test_noalloc_matches_mm_step_on_two_grids_in_a_row():
    big = PU.with_random_start(W.waveguide256(seed=2, steps=40, n=(96, 24, 16)), seed=5, amp_e=1e6, amp_h=2e4)
    it = _run(big, "fp64", 2, 25, 8)
    assert max(it) >= 2                  # the iterations really ran
    small = PU.with_random_start(W.slab64(steps=20), seed=6, amp_e=1e6, amp_h=2e4)
    it = _run(small, "fp64", 1, 12, 4)
    assert max(it) >= 2


def test_noalloc_matches_mm_step_fp32():
    cfg = PU.with_random_start(W.slab64(steps=20), seed=7, amp_e=1e6, amp_h=2e4)
    _run(cfg, "fp32", 1, 10, 3)


def test_noalloc_refusals_enqueue_nothing():
    import paper_2103_12819_amd as mm
    from paper_2103_12819_amd import _native as N
    cfg = W.slab64(steps=4)
    sim = mm.from_config(cfg)            # probes registered, no mm_step yet
    assert _noalloc(sim, 1) == N.MM_ESTATE
    assert b"probes" in sim._lib.mm_last_error(sim._ctx)
    sim.step(1)
    assert _noalloc(sim, 10 ** 6) == N.MM_EINVAL
    assert b"storage" in sim._lib.mm_last_error(sim._ctx)
    assert _noalloc(sim, -1) == N.MM_EINVAL
    assert _noalloc(sim, 0) == 0
    assert list(sim.stats()) == [1, 1]   # nothing ran
    sim.close()
    cfg = W.slab64(steps=4)
    cfg.max_iter = 10 ** 5               # 2 x (1e5 + 2) partials per block: above 4 MiB
    big_iter = mm.from_config(cfg)
    big_iter.step(1)
    assert _noalloc(big_iter, 1) == N.MM_EINVAL
    assert b"4194304" in big_iter._lib.mm_last_error(big_iter._ctx)
    big_iter.close()
