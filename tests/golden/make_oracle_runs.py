"""Write the stored oracle results of the long parity runs.

Runs the FP64 oracle (and nothing else: no HIP code is loaded) on seeded
workloads for their full course and stores what the GPU tests compare with:

  * the iteration count of every H-M sub-step (Sec. 3.2.2 stopping rule),
  * every probe series and probe integral, as exact hexadecimal floats,
  * per field (E, H and the nine M components): the SHA-256 of its FP64
    values (negative zeros folded to +0), its 2-norm, and a seeded sample of
    values for diagnostics.

Runs (the workload builders are the seeded input generators shared by both
sides; they hold none of the method's arithmetic):

  waveguide256   256 x 64 x 64 PEC guide, ferrite slab on the floor, TE10-like
                 port, 2000 steps, flux planes x = 32 and 224
  filter_crop    128 x 64 x 64 crop of the filter grid (two-bar ferrite,
                 dielectric and lossy boxes), 1000 steps

Usage: OMP_NUM_THREADS=1 python tests/golden/make_oracle_runs.py NAME [...]
(about 20 min for waveguide256 and 5 min for filter_crop on one core).
"""
from __future__ import annotations

import gzip
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import from_config  # noqa: E402

FIELDS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz") + tuple("M" + f + c for f in "xyz" for c in "xyz")
N_SAMPLE = 512

RUNS = {
    "waveguide256": lambda: W.waveguide256(seed=0, steps=2000),
    "filter_crop": lambda: W.filter_crop(seed=0, steps=1000),
}


def field_digest(a: np.ndarray) -> str:
    """SHA-256 of the FP64 values in C order, with -0.0 folded to +0.0."""
    v = np.ascontiguousarray(np.asarray(a, dtype=np.float64) + 0.0)
    return hashlib.sha256(v.tobytes()).hexdigest()


def sample_index(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, int(np.prod(shape)), size=N_SAMPLE)


def run(name: str) -> str:
    cfg = RUNS[name]()
    sim = from_config(cfg)
    t0 = time.time()
    chunk = 100
    done = 0
    while done < cfg.steps:
        k = min(chunk, cfg.steps - done)
        sim.step(k)
        done += k
        print(f"{name}: {done}/{cfg.steps} steps, {time.time() - t0:.0f} s", flush=True)
    out = {
        "source": "FP64 oracle (oracle/), written by tests/golden/make_oracle_runs.py",
        "workload": name, "n": list(cfg.n), "steps": cfg.steps, "seed": 0,
        "iters": [int(r) for r in sim.iters],
        "probes": [], "fields": {},
    }
    for pid in range(len(cfg.probes)):
        s = sim.probe_series(pid)
        out["probes"].append({"series": [float(v).hex() for v in s],
                              "sum": float(sim.probe_integral(pid)).hex()})
    for q, nm in enumerate(FIELDS):
        a = np.asarray(sim.field(nm), dtype=np.float64)
        idx = sample_index(a.shape, 1000 + q)
        out["fields"][nm] = {"shape": list(a.shape), "sha256": field_digest(a),
                             "norm": float(np.linalg.norm(a)).hex(),
                             "sample_idx": [int(v) for v in idx],
                             "sample": [float(v).hex() for v in a.reshape(-1)[idx]]}
    path = os.path.join(HERE, f"{name}_oracle.json.gz")
    with gzip.GzipFile(path, "wb", mtime=0) as fh:
        fh.write(json.dumps(out).encode())
    print(f"wrote {path} ({time.time() - t0:.0f} s)", flush=True)
    return path


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(RUNS):
        run(nm)
