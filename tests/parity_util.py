"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare element by element."""
import math

import numpy as np

import workloads as W
from oracle import from_config as oracle_from_config

E_H = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
M_NAMES = tuple("M" + f + c for f in "xyz" for c in "xyz")


def rel_l2(a, b):
    den = float(np.linalg.norm(b))
    num = float(np.linalg.norm(a - b))
    return num / den if den > 0 else num


def run_pair(cfg, steps, precision="fp64", fixed_iter=0, sim_kw=None):
    """Run oracle and HIP path for `steps` steps from the same config.
    Returns (oracle, gpu, oracle_initial) — the last for the M deviations."""
    import paper_2103_12819_amd as mm

    ref = oracle_from_config(cfg, fixed_iter=fixed_iter)
    ref0 = oracle_from_config(cfg, fixed_iter=fixed_iter, with_probes=False)
    ref.step(steps)
    sim = mm.from_config(cfg, precision=precision, fixed_iter=fixed_iter, **(sim_kw or {}))
    sim.step(steps)
    return ref, sim, ref0


def normwise(gpu_parts, ref_parts):
    """||x - y|| / ||y|| over all components of a vector field jointly."""
    num = math.sqrt(sum(float(np.linalg.norm(a - b)) ** 2 for a, b in zip(gpu_parts, ref_parts)))
    den = math.sqrt(sum(float(np.linalg.norm(b)) ** 2 for b in ref_parts))
    return num / den if den > 0 else num


EPS64 = 2.220446049250313e-16


def compare(ref, sim, ref0, tol, check_iters=True, probes=True, dev_tol=None):
    """Normwise relative L2 of E, H, M (all nine components) and normal B,
    and of every probe series / probe integral; all must be <= `tol`.

    The M deviation M - M0 is also compared; its bar is `tol` raised to the
    resolution of FP64 storage of M: an error of ~1000 ulps of |M| in M
    itself, i.e. 1e3 * eps * ||M|| / ||M - M0||.  Per-component errors are
    returned for information."""
    errs, info = {}, {}
    groups = {"E": ("Ex", "Ey", "Ez"), "H": ("Hx", "Hy", "Hz"), "M": M_NAMES, "B": ("Bx", "By", "Bz")}
    got = {nm: sim.field(nm) for g in groups.values() for nm in g}
    exp = {nm: ref.field(nm) for g in groups.values() for nm in g}
    for gname, names in groups.items():
        errs[gname] = normwise([got[n] for n in names], [exp[n] for n in names])
        for n in names:
            info[n] = rel_l2(got[n], exp[n])
    m0 = {n: ref0.field(n) for n in M_NAMES}
    dev_ref = [exp[n] - m0[n] for n in M_NAMES]
    dev_got = [got[n] - m0[n] for n in M_NAMES]
    dnorm = math.sqrt(sum(float(np.linalg.norm(v)) ** 2 for v in dev_ref))
    mnorm = math.sqrt(sum(float(np.linalg.norm(exp[n])) ** 2 for n in M_NAMES))
    dev_err = normwise(dev_got, dev_ref)
    floor = 1e3 * EPS64 * mnorm / dnorm if dnorm > 0 else 0.0
    dev_bar = max(tol if dev_tol is None else dev_tol, floor)
    if probes:
        for pid in range(len(ref.probes)):
            s_gpu, S_gpu = sim.probe(pid)
            s_ref = ref.probe_series(pid)
            assert s_gpu.shape == s_ref.shape
            errs[f"probe{pid}"] = rel_l2(s_gpu, s_ref)
            S_ref = ref.probe_integral(pid)
            scale = max(abs(S_ref), ref.dt * float(np.sum(np.abs(s_ref))), 1e-300)
            errs[f"sum{pid}"] = abs(S_gpu - S_ref) / scale
    bad = {k: v for k, v in errs.items() if not (v <= tol)}
    assert not bad, f"above {tol}: {bad}; per component {info}"
    assert dev_err <= dev_bar or (dnorm == 0 and dev_err == 0), (dev_err, dev_bar)
    if check_iters:
        it = sim.stats()
        assert list(it) == list(ref.iters), (list(it)[:20], ref.iters[:20])
    errs["M_dev"] = dev_err
    errs["M_dev_bar"] = dev_bar
    return errs, info


def with_random_start(cfg, seed, amp_e, amp_h):
    E, H = W.random_fields(cfg, seed=seed, amp_e=amp_e, amp_h=amp_h)
    cfg.E_init, cfg.H_init = E, H
    return cfg
