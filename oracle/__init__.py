"""FP64 CPU oracle for the Neel-rotation Fokker-Planck model.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  The product library (paper_2106_08040_amd) never
imports or calls anything here and shares no code with it.
"""
from .fp_oracle import *  # noqa: F401,F403
from . import mlp_oracle  # noqa: F401,E402
from . import fit_oracle  # noqa: F401,E402
from . import fv_oracle  # noqa: F401,E402
