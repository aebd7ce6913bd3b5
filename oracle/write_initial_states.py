"""Write the initial-state table used by the synthetic workloads
(paper_2510_27447_amd/data/initial_states.json).

LR91: the resting state X* (F(X*) = 0) computed by the oracle's Newton solve.
TT06: the epicardial initial conditions printed with the cell-model
publication (the quiescent state of a paced cell; see oracle.rest).
Run:  python -m oracle.write_initial_states
"""
from __future__ import annotations

import json
import os

from . import rest, tt06
from .models import LR91, TT06

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2510_27447_amd", "data", "initial_states.json")


def table():
    return {
        "_provenance": "written by python -m oracle.write_initial_states; LR91 = oracle rest "
                       "state (F(X*)=0, paper conductances), TT06 = published epicardial "
                       "initial conditions",
        "LR91": dict(zip(LR91.state_names, [float(v) for v in rest.lr91_rest()])),
        "TT06": dict(zip(TT06.state_names, [float(v) for v in tt06.published_initial()])),
    }


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(table(), f, indent=1)
        f.write("\n")
    print("wrote", OUT)
