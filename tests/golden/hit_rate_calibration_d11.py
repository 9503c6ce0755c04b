"""Writes hit_rates_d11.txt: the calibrated rate at which the oracle's decoder
reaches the exact minimum energy (Eqs. (18)-(21)) at the benchmark distance:
rotated d = 11, eta = 100, p in {0.10, 0.15, 0.20, 0.25}, 32 replicas, 2000
sweeps of the geometric schedule 0.05 -> 10.  The exact coset minima come from
the test-side frontier program (tests/_exact_dp.c).  Calls the oracle and that
program only.

    python tests/golden/hit_rate_calibration_d11.py [n_per_p] [threads]
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from tests import _exact  # noqa: E402

CAL_SEED = 911
PS = (0.10, 0.15, 0.20, 0.25)
GREEDY_SEED, ANNEAL_SEED = 21, 22


def hit(job):
    """(hit, class agrees) of one seeded syndrome at noise p."""
    p, i = job
    L = O.Lattice(O.ROTATED, 11)
    pxyz = O.noise(p, 100.0)
    w, wg = O.weights(p, pxyz)
    u = np.random.default_rng([CAL_SEED, int(round(p * 100)), i]).random(L.nq)
    err = np.zeros(L.nq, np.uint8)
    err[u < pxyz[0] + pxyz[1] + pxyz[2]] = 1
    err[u < pxyz[0] + pxyz[1]] = 3
    err[u < pxyz[0]] = 2
    r = L.decode(w, wg, L.syndrome(err), i, 32, O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, 2000), GREEDY_SEED,
                 ANNEAL_SEED)
    exact = [_exact.coset_minimum_c(L.fq, L.fm, r["refs"][0] ^ L.logical(P), w) for P in range(4)]
    assert all(r["e_cls"][P] >= exact[P] for P in range(4)), "E_P below the exact coset minimum"
    return r["e_best"] == min(exact)


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 500
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    lines = ["# Hits of the oracle's decoder at the exact minimum energy (E_best = min over cosets of the",
             "# frontier program's minima), rotated d = 11, eta = 100, 32 replicas, 2000 sweeps geometric",
             f"# 0.05 -> 10, greedy seed {GREEDY_SEED}, anneal seed {ANNEAL_SEED}, syndromes from "
             f"default_rng([{CAL_SEED}, 100 p, index]), uid = index.",
             "# case hits n"]
    with ThreadPoolExecutor(threads) as ex:
        for p in PS:
            h = sum(ex.map(hit, [(p, i) for i in range(n)]))
            lines.append(f"rotated_d11_p{p:.2f} {int(h)} {n}")
            print(lines[-1], flush=True)
    with open(os.path.join(HERE, "hit_rates_d11.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
