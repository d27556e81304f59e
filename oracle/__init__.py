"""FP64 CPU oracle of the coupled Maxwell-LLG step.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark; the product path never imports it.
"""
from .yee_llg import Simulation, from_config, MU0, EPS0, NonConvergence  # noqa: F401
