"""FP64 CPU oracle (test infrastructure only; see likelihood.py and chain.py)."""
from .likelihood import *  # noqa: F401,F403
from .likelihood import evaluate_problem  # noqa: F401
from .chain import branch_lengths_from_time_tree, branch_set_sums, time_tree_gradients  # noqa: F401
