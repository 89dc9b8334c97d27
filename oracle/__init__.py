"""FP64 CPU oracle (test infrastructure only; see tfmm_oracle)."""
from .tfmm_oracle import *  # noqa: F401,F403
