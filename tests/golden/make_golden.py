"""Write the stored oracle tables under tests/golden/.

Calls only the oracle.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import su3ref  # noqa: E402


def m1_plaquette_table():
    """8^4 PBC, beta = 5.7, cold start, 32 sweeps, seed 1, 1-hit: plaquette after each sweep."""
    lat = su3ref.Oracle(8, nlat=1, seed=1, nhit=1)
    lat.start(False)
    rows = []
    for s in range(32):
        lat.sweep(1, 5.7)
        att, acc = lat.counters()
        rows.append({"sweep": s + 1, "plaquette": float(lat.plaquette()[0]), "attempts": att, "accepts": acc})
    return rows


def dlt_plaquette_table():
    """2 x 4^4 DLT (flip_mask 0x7), beta = 5.7, hot start, 4 sweeps, seed 1: per-layer plaquette."""
    lat = su3ref.Oracle(4, nlat=2, flip_mask=0x7, seed=1)
    lat.start(True)
    rows = []
    for s in range(4):
        lat.sweep(1, 5.7)
        p = lat.plaquette()
        rows.append({"sweep": s + 1, "plaquette": [float(v) for v in p]})
    return rows


def main():
    with open(os.path.join(HERE, "m1_plaquette.json"), "w") as f:
        json.dump({"config": "8^4 PBC, beta=5.7, FP64, cold start, 32 sweeps, Philox seed 1, nhit 1",
                   "written_by": "tests/golden/make_golden.py (oracle only)",
                   "rows": m1_plaquette_table()}, f, indent=1)
    with open(os.path.join(HERE, "dlt_plaquette.json"), "w") as f:
        json.dump({"config": "2x4^4 DLT flip_mask 0x7, beta=5.7, FP64, hot start, 4 sweeps, Philox seed 1",
                   "written_by": "tests/golden/make_golden.py (oracle only)",
                   "rows": dlt_plaquette_table()}, f, indent=1)


if __name__ == "__main__":
    main()
