"""Writes tests/golden/oracle_keys.json: oracle signatures of a few small sets.

Calls only oracle/ (and the seeded generators).  The fixture freezes the bit
pattern of the reading of the paper that the oracle implements, so any later
change to the oracle's arithmetic shows up as a failing test that must be
justified by a passage of the paper.

    python tests/golden/make_oracle_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
from paper_1911_00675_amd import workloads as W  # noqa: E402

CASES = [(v, m, n) for v in (1, 2, 3, 4) for (m, n) in ((2, 1), (16, 5), (64, 40), (256, 100))]


def main():
    O.build()
    out = {"_about": __doc__.strip().splitlines()[0], "seed": 0x5EED, "cases": []}
    for k, (v, m, n) in enumerate(CASES):
        b = W.random_sets(1000 + k, 1, n, n, "pareto")
        ids, w = b.set(0)
        keys = O.sign(v, 0x5EED, m, ids, w)
        out["cases"].append({
            "variant": v, "m": m,
            "ids": [str(int(x)) for x in ids],
            "weights": [float(x).hex() for x in w],
            "keys": [format(int(x), "016x") for x in keys],
        })
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_keys.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
