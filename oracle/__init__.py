"""FP64 CPU oracle (test infrastructure only; see likelihood.py)."""
from .likelihood import *  # noqa: F401,F403
from .likelihood import evaluate_problem  # noqa: F401
