"""FP64 CPU oracle of the anisotropic Heisenberg spin-glass Monte Carlo.

TEST INFRASTRUCTURE ONLY: the plain reference the GPU library is checked
against.  Only tests/, the smoke check and the benchmark's CPU-baseline leg
may import it; the GPU library never does, and the two share no code.
"""
from .oracle import *  # noqa: F401,F403
from .ensemble import OracleEnsemble  # noqa: F401
