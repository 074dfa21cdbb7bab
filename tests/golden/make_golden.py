"""Writes the stored oracle histories under tests/golden/ (run from the repo root:
``python tests/golden/make_golden.py``).  Only the FP64 oracle computes the values; the
inputs come from the seeded generators."""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ghom_oracle as go  # noqa: E402
from paper_1901_06531_amd import synth  # noqa: E402


def sphere16():
    w = synth.workload_sphere16()
    o = go.Oracle(w["shape"])
    o.set_material_neohookean(w["phase"], w["mu"], w["lam"])
    o.set_control(w["mask"])
    o.set_history(w["target"])
    o.set_tolerances(w["newton_tol"], w["cg_tol"])
    recs = go.run_history(o)
    return {
        "_source": "FP64 oracle (oracle/ghom_oracle.py) on the 16^3 centred-sphere neo-Hookean "
                   "cell under full stress control, P11 -> 0.1 in 5 increments",
        "workload": w["name"],
        "newton_tol": w["newton_tol"], "cg_tol": w["cg_tol"],
        "steps": [{"F_avg": list(r.F_avg), "P_avg": list(r.P_avg), "newton_iters": r.newton_iters,
                   "cg_iters": r.cg_iters, "cg_per_newton": r.cg_per_newton} for r in recs],
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "sphere16_history.json"), "w") as f:
        json.dump(sphere16(), f, indent=1)
