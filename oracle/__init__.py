"""FP64 CPU oracle (test infrastructure only; see reference.py)."""
from .reference import *  # noqa: F401,F403
from .reference import BlockFactor, admm_analysis, admm_synthesis  # noqa: F401
