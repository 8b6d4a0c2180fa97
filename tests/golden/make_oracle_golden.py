"""Write the stored oracle outputs used as regression fixtures.

Calls only the FP64 oracle (and the seeded input generator).  The paper
prints no worked example with numbers, so the stored values here are the
oracle's own outputs on the 16-taxon HKY+G4 workload; they guard the oracle
against accidental change.  Run from the repository root:
    python tests/golden/make_oracle_golden.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import oracle  # noqa: E402
from paper_2303_04390_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

if __name__ == "__main__":
    prob = synth.config_problem("hky16", seed=0)
    out = oracle.evaluate_problem(prob)
    rec = dict(workload="hky16", seed=0, n_tips=16, n_patterns=1000,
               logl=out["logl"], grad=out["grad"].tolist(),
               absgrad=out["absgrad"].tolist())
    with open(os.path.join(HERE, "hky16_seed0_oracle.json"), "w") as f:
        json.dump(rec, f, indent=1)
