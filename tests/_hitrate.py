"""How often the oracle's decoder reaches the exact minimum energy.

The statistic: for seeded syndromes of a small lattice, the fraction whose
decoded E_best (the least E_P, Eqs. (18)-(21)) equals the exact minimum over
all four cosets, found by enumerating the stabilizer group (tests/_gf2.py).
A hit is a Bernoulli event per syndrome, so the count is binomial and bars on
it follow from exact binomial bounds at a one-sided tail of ALPHA = 3.17e-5
(the normal law's 4 standard deviations).

Shared by the calibration script (tests/golden/hit_rate_calibration.py, which
writes the calibrated rates) and the oracle tests that check against them.
Everything here calls the oracle and the GF(2) enumeration only.
"""
import numpy as np
from scipy import stats

from oracle import oracle as O
from tests import _gf2

# decoder settings of the statistic: the d = 3 workload's noise and schedule;
# colour sweeps and random-site steps with 2 replicas and 200 sweeps linear
# 0.1 -> 5, ladders of 4 levels from beta 0.5 to 3 with 8 replicas and 100 sweeps
P, ETA, N_REP, N_SWEEPS = 0.15, 10.0, 2, 200
LADDER_REP, LADDER_SWEEPS, LADDER = 8, 100, (4, 0.5, 3.0)
GREEDY_SEED, ANNEAL_SEED = 5, 6
ALPHA = 3.17e-5


def _random_problem(L, pxyz, rng):
    u = rng.random(L.nq)
    err = np.zeros(L.nq, np.uint8)
    err[u < pxyz[0] + pxyz[1] + pxyz[2]] = 1
    err[u < pxyz[0] + pxyz[1]] = 3
    err[u < pxyz[0]] = 2
    return L.syndrome(err)


def hits(layout, d, n_syn, seed, rank_order=O.RANK_DEFAULT, order=O.ORDER_COLOUR, n_sweeps=None):
    """Per-syndrome hits (bool array) of the decoder on n_syn syndromes drawn
    from default_rng(seed); uid = syndrome index.  order: colour sweeps,
    random-site steps or ladders (settings above); n_sweeps overrides the
    number of sweeps (a slower schedule's endpoints are kept)."""
    L = O.Lattice(layout, d)
    L.set_rank_order(rank_order)
    w, wg = O.weights(P, O.noise(P, ETA))
    if order == O.ORDER_LADDER:
        beta, n_rep, kw = O.schedule(O.SCHED_LINEAR, 1.0, 1.0, n_sweeps or LADDER_SWEEPS), LADDER_REP, dict(ladder=LADDER)
    else:
        beta, n_rep, kw = O.schedule(O.SCHED_LINEAR, 0.1, 5.0, n_sweeps or N_SWEEPS), N_REP, {}
    group = _gf2.group_elements(_gf2.generator_matrix(L.fq, L.fm, L.nq))
    rng = np.random.default_rng(seed)
    pxyz = O.noise(P, ETA)
    out = np.zeros(n_syn, bool)
    for uid in range(n_syn):
        syn = _random_problem(L, pxyz, rng)
        r = L.decode(w, wg, syn, uid, n_rep, beta, GREEDY_SEED, ANNEAL_SEED, order=order, **kw)
        exact = _gf2.coset_minima(group, [r["refs"][0] ^ L.logical(k) for k in range(4)], w)
        for k in range(4):
            assert r["e_cls"][k] >= exact[k], "E_P below the exact coset minimum"
        out[uid] = r["e_best"] == min(exact)
    return out


def lower_bound(hits_cal, n_cal):
    """One-sided Clopper-Pearson lower bound (tail ALPHA) on the hit
    probability from a calibration of n_cal syndromes with hits_cal hits."""
    if hits_cal == 0:
        return 0.0
    return float(stats.beta.ppf(ALPHA, hits_cal, n_cal - hits_cal + 1))


def bar(hits_cal, n_cal, n):
    """Fewest hits a correct decoder shows on n fresh syndromes: at the
    calibration's lower bound p, the largest h with P(Bin(n, p) < h) <= ALPHA."""
    p = lower_bound(hits_cal, n_cal)
    h = int(stats.binom.ppf(ALPHA, n, p))
    while h > 0 and stats.binom.cdf(h - 1, n, p) > ALPHA:
        h -= 1
    return h


def same_rate(hits_a, hits_b):
    """Two-sided exact test that two decoders hit the exact minimum with the
    same probability, from their hits on the same syndromes (McNemar: given
    the discordant syndromes, each is one decoder's alone with probability
    1/2).  Returns (only_a, only_b, p-value)."""
    a, b = np.asarray(hits_a, bool), np.asarray(hits_b, bool)
    only_a, only_b = int(np.count_nonzero(a & ~b)), int(np.count_nonzero(b & ~a))
    if only_a + only_b == 0:
        return only_a, only_b, 1.0
    return only_a, only_b, float(stats.binomtest(only_a, only_a + only_b, 0.5).pvalue)


def unpaired_p(hits_a, n_a, hits_b, n_b):
    """Two-sided p-value that two binomial counts share one probability
    (Fisher's exact test)."""
    return float(stats.fisher_exact([[hits_a, n_a - hits_a], [hits_b, n_b - hits_b]]).pvalue)


def read_calibration(path):
    """{case: (hits, n)} from the calibration file."""
    out = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        case, h, n = line.split()
        out[case] = (int(h), int(n))
    return out
