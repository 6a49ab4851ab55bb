"""FP64 CPU oracle (test infrastructure only)."""
from .os3d_oracle import *  # noqa: F401,F403
from . import os3d_oracle  # noqa: F401
