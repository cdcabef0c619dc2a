"""Writes the oracle regression fixtures in this folder.

Calls only the oracle and the seeded generator:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tabnet  # noqa: E402
from paper_2510_19689_amd import synth  # noqa: E402


def main():
    p, X = synth.workload("hr35", rows=4)
    lo, ag, ms = tabnet.forward(p, X)
    out = {"source": "oracle.tabnet.forward on workload hr35 (weight seed 1001, data seed 2001), first 4 rows",
           "logits": lo.tolist(), "masks_agg": ag.tolist(), "masks_step": ms.tolist()}
    with open(os.path.join(HERE, "hr35_rows4.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
