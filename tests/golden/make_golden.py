"""Writes the stored expected values under tests/golden/ by calling only the oracle.

    python tests/golden/make_golden.py

level_plans.json: the level schedule of Algorithm 1 (level count, round(w^(l/n_l)) sizes and the
10 / 2 iteration rule of Section III-D) for the workload sizes and a few edge sizes.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

SIZES = [(1, 1), (2, 1), (1, 2), (3, 3), (33, 1), (64, 64), (1024, 768), (4096, 3072),
         (2048, 256), (256, 2048), (5657, 2829), (32767, 3), (1000, 999), (65, 17)]


def main():
    plans = [{"W": W, "H": H, "levels": [list(p) for p in oracle.level_plan(W, H)]}
             for W, H in SIZES]
    doc = {"source": "Algorithm 1 level schedule and the Section III-D iteration rule, "
                     "computed by oracle.level_plan",
           "plans": plans}
    with open(os.path.join(HERE, "level_plans.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
