"""Writes hit_rates_d3.txt: the calibrated rate at which the oracle's decoder
reaches the exact minimum energy (Eqs. (18)-(21)) on small lattices, for the
bars of tests/test_oracle_anneal.py.  Calls the oracle and the test-side GF(2)
enumeration only.

    python tests/golden/hit_rate_calibration.py [n_syn]
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from tests import _hitrate  # noqa: E402

CAL_SEED = 909   # disjoint from the tests' seeds
# case: (layout, within-class rank order, step order)
CASES = {
    "rotated_d3": (O.ROTATED, O.RANK_DEFAULT, O.ORDER_COLOUR),
    "planar_d3": (O.PLANAR, O.RANK_DEFAULT, O.ORDER_COLOUR),
    "planar_d3_face_id": (O.PLANAR, O.RANK_FACE_ID, O.ORDER_COLOUR),
    "rotated_d3_site": (O.ROTATED, O.RANK_DEFAULT, O.ORDER_RANDOM_SITE),
    "planar_d3_site": (O.PLANAR, O.RANK_DEFAULT, O.ORDER_RANDOM_SITE),
    "rotated_d3_ladder": (O.ROTATED, O.RANK_DEFAULT, O.ORDER_LADDER),
    "planar_d3_ladder": (O.PLANAR, O.RANK_DEFAULT, O.ORDER_LADDER),
}


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 4000
    lines = ["# Hits of the oracle's decoder at the exact minimum energy (E_best = min over cosets of",
             "# the enumerated minima), d = 3, p = 0.15, eta = 10; colour sweeps and random-site steps:",
             "# 2 replicas, 200 sweeps linear 0.1 -> 5; ladders: 4 levels, beta 0.5 -> 3, 8 replicas,",
             f"# 100 sweeps; greedy seed {_hitrate.GREEDY_SEED}, anneal seed {_hitrate.ANNEAL_SEED}, "
             f"syndromes from default_rng({CAL_SEED}), uid = index.",
             "# planar_d3_face_id: colour sweeps with face-id rank order inside each colour class.",
             "# case hits n"]
    for name, (layout, rank, order) in CASES.items():
        h = _hitrate.hits(layout, 3, n, CAL_SEED, rank, order)
        lines.append(f"{name} {int(h.sum())} {n}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "hit_rates_d3.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
