"""Gradient check at the full design-problem size: 128x64x64 waveguide with a
smooth random eps_r in [1,4] and Ms in [1e5,1.8e5] over a 64x32x16 region,
4000 steps, loss = time-integrated Poynting flux at x = 120, checkpoints
every 100 steps; mm_adjoint against central differences (h = 1e-6
relative) of the HIP forward on 32 random design cells, for eps_r and Ms.
Fixed-iteration mode (3 per sub-step) keeps the forward smooth in the
parameters.  128 forward runs of 4000 steps: about 2 minutes on the GPU."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_design128_gradient_central_differences():
    import paper_2103_12819_amd as mm
    cfg = W.design128(seed=0, steps=4000)
    sim = mm.from_config(cfg, fixed_iter=3)
    sim.enable_adjoint(100)
    sim.step(cfg.steps)
    _, L = sim.probe(0)
    ge, gm = sim.adjoint(0)
    sim.close()
    rng = np.random.default_rng(2)
    cells = [tuple(c) for c in np.argwhere(cfg.Ms > 0)]
    picks = [cells[i] for i in rng.choice(len(cells), 32, replace=False)]
    rows = []
    print(f"design128 central differences on {len(picks)} cells (eps_r and Ms), 4000 steps each", flush=True)
    for idx in picks:
        for which, g, base in (("eps", ge, cfg.eps_r), ("ms", gm, cfg.Ms)):
            h = 1e-6 * base[idx]
            vals = []
            for sgn in (1, -1):
                p = base.copy()
                p[idx] += sgn * h
                c2 = W.design128(seed=0, steps=4000)
                if which == "eps":
                    c2.eps_r = p
                else:
                    c2.Ms = p
                s2 = mm.from_config(c2, fixed_iter=3)
                s2.step(c2.steps)
                vals.append(s2.probe(0)[1])
                s2.close()
            fd = (vals[0] - vals[1]) / (2 * h)
            floor = 1e3 * 2.220446049250313e-16 * abs(L) / h
            rows.append((which, idx, fd, g[idx], floor))
            print(f"  {len(rows)}/{2 * len(picks)} {which} {idx} fd {fd:.6e} adjoint {g[idx]:.6e}", flush=True)
    for which, idx, fd, ad, floor in rows:
        print(f"{which} {idx} fd={fd:.6e} adj={ad:.6e} rel={abs(fd - ad) / max(abs(ad), 1e-300):.2e} "
              f"floor/|adj|={floor / max(abs(ad), 1e-300):.2e}", flush=True)
    for which, idx, fd, ad, floor in rows:
        assert abs(fd - ad) <= 1e-6 * abs(ad) + floor, (which, idx, fd, ad, floor)
