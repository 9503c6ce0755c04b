"""Pins for the oracle's simulated annealing (Algs. 2-3) and decoder (Alg. 7).

Pins: exact coset minima by brute-force enumeration of the stabilizer group
(Eqs. (18)-(21)), the beta = 0 and beta = infinity closed forms, the empty
schedule, per-sweep invariants, the stationary Boltzmann law of Eq. (22) at a
fixed beta (chi-square, with a negative control), and the coset relabelling
of Eqs. (35)-(36).
"""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from tests import _exact, _gf2, _hitrate

# calibrated hit rates at the exact minimum (tests/golden/hit_rate_calibration.py)
CAL = _hitrate.read_calibration(os.path.join(os.path.dirname(__file__), "golden", "hit_rates_d3.txt"))


def random_problem(L, p, eta, rng):
    pxyz = O.noise(p, eta)
    u = rng.random(L.nq)
    err = np.zeros(L.nq, np.uint8)
    err[u < pxyz[0] + pxyz[1] + pxyz[2]] = 1
    err[u < pxyz[0] + pxyz[1]] = 3
    err[u < pxyz[0]] = 2
    return err, L.syndrome(err)


def test_zero_sweeps_returns_initial_energy():
    L = O.Lattice(O.ROTATED, 5)
    w, _ = O.weights(0.1, O.noise(0.1, 3.0))
    rng = np.random.default_rng(1)
    init = rng.integers(0, 4, L.nq).astype(np.uint8)
    r = L.anneal_chain(w, np.zeros(0), 7, 3, 1, init)
    e0 = int(w[init].sum())
    assert r["e"] == r["emin"] == e0 and r["stop"] == 0
    assert np.array_equal(r["final"], init) and np.array_equal(r["snap"], init)


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 3), (O.ROTATED, 7), (O.PLANAR, 5)])
def test_beta_zero_closed_form(layout, d):
    """beta = 0: every proposed flip is accepted (the draw u = 2^32-1, the only
    exception, has probability 2^-32 per move), so phase k of each sweep
    multiplies the configuration by the product of all class-k generators."""
    L = O.Lattice(layout, d)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    cls_prod = [np.bitwise_xor.reduce(G[L.fclass == k], axis=0) for k in range(4)]
    w, _ = O.weights(0.12, O.noise(0.12, 10.0))
    rng = np.random.default_rng(2)
    init = rng.integers(0, 4, L.nq).astype(np.uint8)
    n = 7
    r = L.anneal_chain(w, np.zeros(n), 99, 5, 2, init)
    cfg = init.copy()
    e_min, stop, snap = int(w[cfg].sum()), 0, cfg.copy()
    for t in range(n):
        for k in range(4):
            cfg = cfg ^ cls_prod[k]
            e = int(w[cfg].sum())
            if e < e_min:
                e_min, stop, snap = e, 4 * t + k + 1, cfg.copy()
    assert np.array_equal(r["final"], cfg)
    assert r["e"] == int(w[cfg].sum())
    assert (r["emin"], r["stop"]) == (e_min, stop)
    assert np.array_equal(r["snap"], snap)


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 5), (O.PLANAR, 5)])
def test_zero_temperature_descent(layout, d):
    """beta -> infinity: only moves with dE <= 0 are accepted, so the energy is
    non-increasing sweep by sweep and E_min is the final energy."""
    L = O.Lattice(layout, d)
    w, _ = O.weights(0.15, O.noise(0.15, 10.0))
    rng = np.random.default_rng(3)
    init = rng.integers(0, 4, L.nq).astype(np.uint8)
    beta = np.full(12, 1e6)
    es = [L.anneal_chain(w, beta[:s], 4, 1, 0, init)["e"] for s in range(13)]
    assert all(a >= b for a, b in zip(es, es[1:]))
    r = L.anneal_chain(w, beta, 4, 1, 0, init)
    assert r["emin"] == r["e"] == es[-1] and es[-1] < es[0]


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 5), (O.ROTATED, 9), (O.PLANAR, 5), (O.PLANAR, 7)])
def test_invariants_every_sweep(layout, d):
    """After every sweep: syndrome unchanged, incremental energy equal to the
    recomputed energy (Eq. (10)), coset unchanged, E_min <= E (oracle's check
    mode returns an error code on any violation)."""
    L = O.Lattice(layout, d)
    w, _ = O.weights(0.2, O.noise(0.2, 10.0))
    rng = np.random.default_rng(4)
    beta = O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, 40)
    for c in range(6):
        init = rng.integers(0, 4, L.nq).astype(np.uint8)
        r = L.anneal_chain(w, beta, 17, 8, c, init, check=True)
        assert L.energy(w, r["snap"]) == r["emin"] <= r["e"]
        assert np.array_equal(L.syndrome(r["snap"]), L.syndrome(init))
        assert L.cls(r["snap"], init) == 0 and L.cls(r["final"], init) == 0


def test_boltzmann_law_fixed_beta():
    """Eq. (22): each Metropolis move satisfies detailed balance for
    pi_beta = exp(-beta H), so the class-by-class sweep leaves pi_beta
    stationary.  Final states of many independent chains at a fixed beta are
    compared with the exact law over the 256-element coset (d = 3)."""
    L = O.Lattice(O.ROTATED, 3)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    w, _ = O.weights(0.15, O.noise(0.15, 10.0))
    rng = np.random.default_rng(6)
    init = rng.integers(0, 4, L.nq).astype(np.uint8)
    elems = _gf2.group_elements(G) ^ _gf2.pack(init)
    index = {int(v): i for i, v in enumerate(elems)}
    energies = _gf2.packed_energy(elems, w).astype(np.float64)
    beta = 0.35
    n_chains, n_sweeps = 12000, 25
    counts = np.zeros(len(elems))
    bs = np.full(n_sweeps, beta)
    for c in range(n_chains):
        r = L.anneal_chain(w, bs, 2024, 77, c, init, want_snap=False)
        counts[index[int(_gf2.pack(r["final"]))]] += 1

    def chi2_p(b):
        pr = np.exp(-b * (energies - energies.min()) / 65536.0)
        pr /= pr.sum()
        exp = pr * n_chains
        keep = exp >= 5
        obs = np.append(counts[keep], counts[~keep].sum())
        ex = np.append(exp[keep], exp[~keep].sum())
        if ex[-1] == 0:
            obs, ex = obs[:-1], ex[:-1]
        return stats.chisquare(obs, ex).pvalue

    assert chi2_p(beta) > 1e-3
    # negative control: a beta off by 30 percent is rejected decisively
    assert chi2_p(1.3 * beta) < 1e-6


def _exact_coset_minima(L, w, ref):
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    group = _gf2.group_elements(G)
    return _gf2.coset_minima(group, [ref ^ L.logical(P) for P in range(4)], w)


@pytest.mark.parametrize("layout,d,n_syn,case", [(O.ROTATED, 3, 400, "rotated_d3"), (O.PLANAR, 3, 1000, "planar_d3"),
                                                (O.ROTATED, 5, 3, None)])
def test_decoder_against_brute_force(layout, d, n_syn, case):
    """Eqs. (18)-(21): E_P estimates the exact coset minimum from above; the
    decoder's recovery is syndrome-consistent, has energy E_best and lies in
    coset P* (relative to R_0).  At d = 3 the count of syndromes whose E_best
    is the exact minimum must reach the binomial bar of the calibrated rate
    (tests/_hitrate.py); at d = 5 (three syndromes, 2^24 group elements each)
    only the bounds are checked."""
    L = O.Lattice(layout, d)
    p, eta = 0.15, 10.0
    w, wg = O.weights(p, O.noise(p, eta))
    beta = O.schedule(O.SCHED_LINEAR, 0.1, 5.0, 200)
    rng = np.random.default_rng(10 + d)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    group = _gf2.group_elements(G)
    hits = 0
    for uid in range(n_syn):
        _, syn = random_problem(L, p, eta, rng)
        out = L.decode(w, wg, syn, uid, 2, beta, 5, 6)
        r0 = out["refs"][0]
        exact = _gf2.coset_minima(group, [r0 ^ L.logical(P) for P in range(4)], w)
        for P in range(4):
            assert out["e_cls"][P] >= exact[P]
        assert out["e_best"] == min(out["e_cls"]) >= min(exact)
        assert out["cls"] == int(np.argmin(out["e_cls"]))
        rec = out["recovery"]
        assert np.array_equal(L.syndrome(rec), syn)
        assert L.energy(w, rec) == out["e_best"]
        assert L.cls(rec, r0) == out["cls"]
        assert L.cls(out["paper_recovery"], r0) == out["cls"]
        hits += out["e_best"] == min(exact)
    if case:
        assert hits >= _hitrate.bar(*CAL[case], n_syn)


def test_rank_order_leaves_hit_rate_unchanged():
    """The within-class rank only names the Philox word each generator of a
    colour class draws (Alg. 3 leaves the visiting order open), so the planar
    lattice's two readings -- face-id order and the order of the lattice
    turned by 45 degrees -- must give chains of one law.  Checked on the
    statistic they are tested by: on the same 2000 syndromes the syndromes
    that only one order decodes to the exact minimum split evenly (exact
    McNemar test), each order clears its calibrated bar, and the calibrated
    rates agree (Fisher's exact test).  Negative control: 150 instead of 200
    sweeps, a real loss of quality, is told apart decisively."""
    n = 2000
    a = _hitrate.hits(O.PLANAR, 3, n, 13, O.RANK_DEFAULT)
    b = _hitrate.hits(O.PLANAR, 3, n, 13, O.RANK_FACE_ID)
    assert a.sum() >= _hitrate.bar(*CAL["planar_d3"], n)
    assert b.sum() >= _hitrate.bar(*CAL["planar_d3_face_id"], n)
    only_a, only_b, pv = _hitrate.same_rate(a, b)
    assert pv > _hitrate.ALPHA, (only_a, only_b)
    assert _hitrate.unpaired_p(*CAL["planar_d3"], *CAL["planar_d3_face_id"]) > _hitrate.ALPHA
    worse = _hitrate.hits(O.PLANAR, 3, n, 13, O.RANK_DEFAULT, n_sweeps=150)
    only_a, only_w, pv = _hitrate.same_rate(a, worse)
    assert only_a > only_w and pv < _hitrate.ALPHA


def test_rank_order_hook():
    """The test hook re-ranks every class as a permutation of 0..M-1 (face-id
    order ascending with the face id); the default order is restored."""
    L = O.Lattice(O.PLANAR, 5)
    default = L.frank.copy()
    L.set_rank_order(O.RANK_FACE_ID)
    for k in range(4):
        faces = np.flatnonzero(L.fclass == k)
        assert np.array_equal(L.frank[faces], np.arange(len(faces)))
    assert not np.array_equal(L.frank, default)
    L.set_rank_order(O.RANK_DEFAULT)
    assert np.array_equal(L.frank, default)
    with pytest.raises(ValueError):
        L.set_rank_order(7)


def test_coset_relabelling():
    """Eqs. (35)-(36): Q_r = [R_r R_0] and chain (r, P) estimates coset Q_r P;
    checked with an independent symplectic computation of the class."""
    L = O.Lattice(O.ROTATED, 7)
    p, eta = 0.2, 10.0
    w, wg = O.weights(p, O.noise(p, eta))
    rng = np.random.default_rng(8)
    _, syn = random_problem(L, p, eta, rng)
    out = L.decode(w, wg, syn, 3, 8, O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, 20), 1, 2, chains=True)
    refs = out["refs"]
    logs = np.stack([L.lx, L.lz])
    for r in range(8):
        e = refs[r] ^ refs[0]
        a, b = _gf2.symp_products(e[None], logs)[0]  # vs L_X, vs L_Z
        expect = {(0, 0): 0, (0, 1): 1, (1, 1): 2, (1, 0): 3}[(int(a), int(b))]
        assert out["qcls"][r] == expect
        for P in range(4):
            fin = out["chain_final"][4 * r + P]
            assert np.array_equal(L.syndrome(fin), syn)
            assert L.cls(fin, refs[0]) == O.lib().or_class_mul(expect, P)


# --- the literal random-site chain (Alg. 3 as printed) -------------------------

SITE = O.ORDER_RANDOM_SITE


def test_site_draw_bins():
    """The site of a 32-bit draw u is floor(u N / 2^32): the draws that pick
    generator f are the u in [ceil(f 2^32 / N), ceil((f + 1) 2^32 / N)), so
    every generator gets the same number of draws up to one (uniform within
    N / 2^32)."""
    for n in (8, 24, 120, 144, 960):
        starts = [-((-f << 32) // n) for f in range(n + 1)]   # ceil(f 2^32 / n)
        sizes = np.diff(starts)
        assert sizes.max() - sizes.min() <= 1
        for f in range(n):
            assert O.site_of(starts[f], n) == f
            assert O.site_of(starts[f + 1] - 1, n) == f


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 3), (O.ROTATED, 7), (O.PLANAR, 5)])
def test_site_beta_zero_closed_form(layout, d):
    """beta = 0: every step's move is accepted (u_a = 2^32-1 aside, probability
    2^-32), so step m of sweep t multiplies by the generator its Philox site
    draw names (block (uid, c, 2^31 + t, m div 2), word 2(m mod 2)); E_min
    and its step are tracked after every step (Alg. 2)."""
    L = O.Lattice(layout, d)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    w, _ = O.weights(0.12, O.noise(0.12, 10.0))
    rng = np.random.default_rng(12)
    init = rng.integers(0, 4, L.nq).astype(np.uint8)
    seed, uid, chain, n = 0xABCDEF0123, 5, 6, 3
    r = L.anneal_chain(w, np.zeros(n), seed, uid, chain, init, order=SITE)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    cfg = init.copy()
    e_min, stop, snap = int(w[cfg].sum()), 0, cfg.copy()
    for t in range(n):
        for m in range(L.nstab):
            block = O.philox((uid, chain, 0x80000000 + t, m >> 1), key)
            f = O.site_of(block[2 * (m & 1)], L.nstab)
            cfg = cfg ^ G[f]
            e = int(w[cfg].sum())
            if e < e_min:
                e_min, stop, snap = e, t * L.nstab + m + 1, cfg.copy()
    assert np.array_equal(r["final"], cfg)
    assert r["e"] == int(w[cfg].sum())
    assert (r["emin"], r["stop"]) == (e_min, stop)
    assert np.array_equal(r["snap"], snap)


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 5), (O.PLANAR, 5)])
def test_site_zero_temperature_descent(layout, d):
    L = O.Lattice(layout, d)
    w, _ = O.weights(0.15, O.noise(0.15, 10.0))
    rng = np.random.default_rng(13)
    init = rng.integers(0, 4, L.nq).astype(np.uint8)
    beta = np.full(12, 1e6)
    es = [L.anneal_chain(w, beta[:s], 4, 1, 0, init, order=SITE)["e"] for s in range(13)]
    assert all(a >= b for a, b in zip(es, es[1:]))
    r = L.anneal_chain(w, beta, 4, 1, 0, init, order=SITE)
    assert r["emin"] == r["e"] == es[-1] and es[-1] < es[0]


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 5), (O.ROTATED, 9), (O.PLANAR, 7)])
def test_site_invariants_every_sweep(layout, d):
    L = O.Lattice(layout, d)
    w, _ = O.weights(0.2, O.noise(0.2, 10.0))
    rng = np.random.default_rng(14)
    beta = O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, 40)
    for c in range(6):
        init = rng.integers(0, 4, L.nq).astype(np.uint8)
        r = L.anneal_chain(w, beta, 17, 8, c, init, check=True, order=SITE)
        assert L.energy(w, r["snap"]) == r["emin"] <= r["e"]
        assert np.array_equal(L.syndrome(r["snap"]), L.syndrome(init))
        assert L.cls(r["snap"], init) == 0 and L.cls(r["final"], init) == 0


def test_site_boltzmann_law_fixed_beta():
    """A uniformly chosen generator is a symmetric proposal (each G_f is its
    own inverse), so each random-site step satisfies detailed balance for
    pi_beta of Eq. (22); final states of independent chains at a fixed beta
    follow the exact law over the 256-element coset (d = 3).  From this
    start the two degenerate ground states are separated by a barrier, so the
    chains run 100 sweeps (25 do not mix for either sweep order)."""
    L = O.Lattice(O.ROTATED, 3)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    w, _ = O.weights(0.15, O.noise(0.15, 10.0))
    rng = np.random.default_rng(16)
    init = rng.integers(0, 4, L.nq).astype(np.uint8)
    elems = _gf2.group_elements(G) ^ _gf2.pack(init)
    index = {int(v): i for i, v in enumerate(elems)}
    energies = _gf2.packed_energy(elems, w).astype(np.float64)
    beta = 0.35
    n_chains, n_sweeps = 8000, 100
    counts = np.zeros(len(elems))
    bs = np.full(n_sweeps, beta)
    for c in range(n_chains):
        r = L.anneal_chain(w, bs, 2025, 78, c, init, want_snap=False, order=SITE)
        counts[index[int(_gf2.pack(r["final"]))]] += 1

    def chi2_p(b):
        pr = np.exp(-b * (energies - energies.min()) / 65536.0)
        pr /= pr.sum()
        exp = pr * n_chains
        keep = exp >= 5
        obs = np.append(counts[keep], counts[~keep].sum())
        ex = np.append(exp[keep], exp[~keep].sum())
        if ex[-1] == 0:
            obs, ex = obs[:-1], ex[:-1]
        return stats.chisquare(obs, ex).pvalue

    assert chi2_p(beta) > 1e-3
    assert chi2_p(1.3 * beta) < 1e-6


@pytest.mark.parametrize("layout,d,n_syn,case", [(O.ROTATED, 3, 400, "rotated_d3_site"),
                                                (O.PLANAR, 3, 400, "planar_d3_site")])
def test_site_decoder_against_brute_force(layout, d, n_syn, case):
    """The decoder on random-site chains: E_P bounds the exact coset minimum
    from above, the recovery is consistent, and the count of syndromes decoded
    to the exact minimum reaches the calibrated binomial bar."""
    L = O.Lattice(layout, d)
    p, eta = 0.15, 10.0
    w, wg = O.weights(p, O.noise(p, eta))
    beta = O.schedule(O.SCHED_LINEAR, 0.1, 5.0, 200)
    rng = np.random.default_rng(20 + d)
    hits = 0
    for uid in range(n_syn):
        _, syn = random_problem(L, p, eta, rng)
        out = L.decode(w, wg, syn, uid, 2, beta, 5, 6, order=SITE, chains=True)
        r0 = out["refs"][0]
        exact = _exact_coset_minima(L, w, r0)
        for P in range(4):
            assert out["e_cls"][P] >= exact[P]
        assert out["e_best"] == min(out["e_cls"])
        rec = out["recovery"]
        assert np.array_equal(L.syndrome(rec), syn)
        assert L.energy(w, rec) == out["e_best"]
        assert L.cls(rec, r0) == out["cls"]
        assert out["chain_stop"].max() <= len(beta) * L.nstab
        hits += out["e_best"] == min(exact)
    assert hits >= _hitrate.bar(*CAL[case], n_syn)


# --- replica exchange (ladders of fixed inverse temperatures) -------------------

LADDER = O.ORDER_LADDER


@pytest.mark.parametrize("delta", [0.05, 0.5, 3.0])
def test_swap_threshold_closed_form(delta):
    """T(n) is floor(2^32 exp(-delta n 2^-16)) up to the truncations of the
    fixed-point product (relative error below n 2^-50 + 2^-58) and one unit."""
    R = O.swap_powers(delta)
    rng = np.random.default_rng(30)
    ns = [1, 2, 3, 255, 65536, 1 << 20, (1 << 31) - 1] + rng.integers(1, 1 << 24, 200).tolist()
    for n in ns:
        exact = 2.0 ** 32 * np.exp(-delta * n / 65536.0)
        tol = exact * (n * 2.0 ** -50 + 2.0 ** -58) + 1.0
        assert abs(O.swap_threshold(R, n) - exact) <= tol, n
    # delta = 0: every exchange accepted but for the top few draws
    R0 = O.swap_powers(0.0)
    assert all(O.swap_threshold(R0, n) >= 2 ** 32 - 64 for n in (1, 1000, (1 << 31) - 1))


def test_ladder_of_one_is_a_constant_beta_chain():
    """K = 1: the ladder's only chain is the colour-sweep chain at the constant
    beta_lo, draw for draw."""
    L = O.Lattice(O.ROTATED, 5)
    w, _ = O.weights(0.15, O.noise(0.15, 10.0))
    rng = np.random.default_rng(31)
    init = rng.integers(0, 4, L.nq).astype(np.uint8)
    lad = L.anneal_ladder(w, 0.7, 0.7, 1, 30, 11, 5, 2, [9], init[None])
    ref = L.anneal_chain(w, np.full(30, 0.7), 11, 5, 9, init)
    assert lad["e"][0] == ref["e"] and lad["emin"][0] == ref["emin"] and lad["stop"][0] == ref["stop"]
    assert np.array_equal(lad["final"][0], ref["final"]) and np.array_equal(lad["snap"][0], ref["snap"])


def test_ladder_of_equal_levels():
    """beta_lo = beta_hi: every level sweeps at the same beta, so each chain is
    the constant-beta chain of its own id, and every exchange is accepted:
    the levels follow the alternating even/odd transpositions."""
    L = O.Lattice(O.PLANAR, 5)
    w, _ = O.weights(0.15, O.noise(0.15, 5.0, 1))
    rng = np.random.default_rng(32)
    init = rng.integers(0, 4, (4, L.nq)).astype(np.uint8)
    ids = [3, 7, 11, 15]
    n = 9
    lad = L.anneal_ladder(w, 0.8, 0.8, 4, n, 12, 6, 3, ids, init)
    for j in range(4):
        ref = L.anneal_chain(w, np.full(n, 0.8), 12, 6, ids[j], init[j])
        assert (lad["e"][j], lad["emin"][j], lad["stop"][j]) == (ref["e"], ref["emin"], ref["stop"])
        assert np.array_equal(lad["final"][j], ref["final"])
    level = list(range(4))
    for t in range(n):
        for k in range(t & 1, 3, 2):
            lo, hi = level.index(k), level.index(k + 1)
            level[lo], level[hi] = k + 1, k
    assert lad["level"].tolist() == level


def test_ladder_boltzmann_law():
    """Each level's sweep leaves pi_beta of Eq. (22) stationary and the
    exchange satisfies detailed balance for the product law over levels, so
    the chain at each level of many independent two-level ladders follows the
    exact law at that level's beta over the 256-element coset (d = 3)."""
    L = O.Lattice(O.ROTATED, 3)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    w, _ = O.weights(0.15, O.noise(0.15, 10.0))
    rng = np.random.default_rng(33)
    init = rng.integers(0, 4, L.nq).astype(np.uint8)
    elems = _gf2.group_elements(G) ^ _gf2.pack(init)
    index = {int(v): i for i, v in enumerate(elems)}
    energies = _gf2.packed_energy(elems, w).astype(np.float64)
    betas = (0.15, 0.45)
    n_ladders, n_sweeps = 6000, 60
    counts = np.zeros((2, len(elems)))
    for c in range(n_ladders):
        r = L.anneal_ladder(w, betas[0], betas[1], 2, n_sweeps, 2026, 79, c, [2 * c, 2 * c + 1],
                            np.stack([init, init]), want_snap=False)
        for j in range(2):
            counts[r["level"][j], index[int(_gf2.pack(r["final"][j]))]] += 1

    def chi2_p(level, b):
        pr = np.exp(-b * (energies - energies.min()) / 65536.0)
        pr /= pr.sum()
        exp = pr * n_ladders
        keep = exp >= 5
        obs = np.append(counts[level][keep], counts[level][~keep].sum())
        ex = np.append(exp[keep], exp[~keep].sum())
        if ex[-1] == 0:
            obs, ex = obs[:-1], ex[:-1]
        return stats.chisquare(obs, ex).pvalue

    assert chi2_p(0, betas[0]) > 1e-3 and chi2_p(1, betas[1]) > 1e-3
    # negative controls: the two levels' laws are told apart decisively
    assert chi2_p(1, betas[0]) < 1e-6 and chi2_p(0, betas[1]) < 1e-6


@pytest.mark.parametrize("layout,d,n_syn,case", [(O.ROTATED, 3, 200, "rotated_d3_ladder"),
                                                (O.PLANAR, 3, 200, "planar_d3_ladder")])
def test_ladder_decoder_against_brute_force(layout, d, n_syn, case):
    """The decoder on ladders (K = 4 levels from beta 0.5 to 3): replicas of a
    ladder share one greedy reference, E_P bounds the exact coset minimum from
    above, the recovery is consistent, and the count of syndromes decoded to
    the exact minimum reaches the calibrated binomial bar."""
    L = O.Lattice(layout, d)
    p, eta = 0.15, 10.0
    w, wg = O.weights(p, O.noise(p, eta))
    rng = np.random.default_rng(40 + d)
    hits = 0
    for uid in range(n_syn):
        _, syn = random_problem(L, p, eta, rng)
        out = L.decode(w, wg, syn, uid, 8, np.ones(100), 5, 6, order=LADDER, ladder=(4, 0.5, 3.0), chains=True)
        refs = out["refs"]
        assert all(np.array_equal(refs[r], refs[4 * (r // 4)]) for r in range(8))
        r0 = refs[0]
        exact = _exact_coset_minima(L, w, r0)
        for P in range(4):
            assert out["e_cls"][P] >= exact[P]
        assert out["e_best"] == min(out["e_cls"])
        rec = out["recovery"]
        assert np.array_equal(L.syndrome(rec), syn)
        assert L.energy(w, rec) == out["e_best"]
        assert L.cls(rec, r0) == out["cls"]
        hits += out["e_best"] == min(exact)
    assert hits >= _hitrate.bar(*CAL[case], n_syn)


# --- exact coset minima beyond brute force (frontier dynamic program) ----------

@pytest.mark.parametrize("layout,d", [(O.ROTATED, 3), (O.PLANAR, 3), (O.ROTATED, 5)])
def test_frontier_program_equals_brute_force(layout, d):
    """The exact minimiser used below agrees with enumeration of the whole
    stabilizer group where that is feasible."""
    L = O.Lattice(layout, d)
    w, _ = O.weights(0.15, O.noise(0.15, 10.0))
    rng = np.random.default_rng(50 + d)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    group = _gf2.group_elements(G)
    for _ in range(3):
        c0 = rng.integers(0, 4, L.nq).astype(np.uint8)
        exact = _gf2.coset_minima(group, [c0], w)[0]
        assert _exact.coset_minimum(L.fq, L.fm, c0, w) == exact


@pytest.mark.parametrize("layout,d,n_syn", [(O.ROTATED, 7, 4), (O.PLANAR, 5, 4)])
def test_decoder_against_exact_minima(layout, d, n_syn):
    """Beyond brute force: E_P bounds the exact coset minimum from above for
    every coset, and a slow schedule reaches the exact least coset minimum."""
    L = O.Lattice(layout, d)
    p, eta = 0.12, 10.0
    w, wg = O.weights(p, O.noise(p, eta))
    beta = O.schedule(O.SCHED_LINEAR, 0.1, 5.0, 400)
    rng = np.random.default_rng(60 + d)
    hits = 0
    for uid in range(n_syn):
        _, syn = random_problem(L, p, eta, rng)
        out = L.decode(w, wg, syn, uid, 4, beta, 5, 6)
        r0 = out["refs"][0]
        exact = [_exact.coset_minimum(L.fq, L.fm, r0 ^ L.logical(P), w) for P in range(4)]
        for P in range(4):
            assert out["e_cls"][P] >= exact[P]
        hits += out["e_best"] == min(exact)
    assert hits >= n_syn - 1


@pytest.mark.parametrize("layout,d,n_rep,mode", [(O.ROTATED, 5, 4, O.GREEDY_RANDOM), (O.PLANAR, 5, 3, O.GREEDY_RANDOM),
                                                 (O.ROTATED, 7, 2, O.GREEDY_SAME)])
def test_selection_by_chain_equals_decode(layout, d, n_rep, mode):
    """Alg. 7's selection (Eq. (21)) run after the chains, as the tests do to
    spread one large syndrome's chains over host threads, equals the oracle's
    decode, which selects as it goes: E_P, P*, the best chain and its
    snapshot.  Also the reading of ties: E_P of an empty coset is the largest
    value, and P* and the best chain go to the lowest index."""
    from tests._parity import oracle_decode_by_chain
    L = O.Lattice(layout, d)
    p, eta = 0.15, 10.0
    w, wg = O.weights(p, O.noise(p, eta))
    beta = O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, 30)
    rng = np.random.default_rng(90 + d)
    for uid in range(6):
        _, syn = random_problem(L, p, eta, rng)
        a = L.decode(w, wg, syn, uid, n_rep, beta, 11, 12, greedy_mode=mode, chains=True)
        if mode == O.GREEDY_SAME:
            continue   # the helper draws randomized references
        b = oracle_decode_by_chain(layout, d, w, wg, syn, uid, n_rep, beta, 11, 12)
        for k in ("refs", "qcls", "chain_emin", "chain_stop", "chain_e", "e_cls", "recovery"):
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
        for k in ("cls", "e_best", "best_chain"):
            assert a[k] == b[k], k
    big = np.iinfo(np.int64).max
    e_cls, ps, bc = O.reduce(np.array([9, 4, 4, 7, 4]), np.array([0, 1, 3, 1, 1]))
    assert list(e_cls) == [9, 4, big, 4] and ps == 1 and bc == 1
    with pytest.raises(ValueError):
        O.reduce(np.array([1]), np.array([4]))


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 3), (O.PLANAR, 3), (O.ROTATED, 5), (O.ROTATED, 7), (O.PLANAR, 5)])
def test_frontier_program_in_c(layout, d):
    """The C form of the frontier program (used at d = 11) equals the Python
    one, and enumeration of the stabilizer group where that is feasible."""
    L = O.Lattice(layout, d)
    rng = np.random.default_rng(70 + d + 10 * layout)
    group = _gf2.group_elements(_gf2.generator_matrix(L.fq, L.fm, L.nq)) if L.nstab <= 16 else None
    for k in range(3):
        p, eta = float(rng.uniform(0.05, 0.3)), float(10 ** rng.uniform(0, 3))
        w, _ = O.weights(p, O.noise(p, eta))
        c0 = rng.integers(0, 4, L.nq).astype(np.uint8)
        got = _exact.coset_minimum_c(L.fq, L.fm, c0, w)
        assert got == _exact.coset_minimum(L.fq, L.fm, c0, w)
        if group is not None:
            assert got == _gf2.coset_minima(group, [c0], w)[0]


def test_decoder_against_exact_minima_d11():
    """At the benchmark distance (rotated d = 11, eta = 100, 32 replicas, 2000
    sweeps of the geometric schedule 0.05 -> 10): every E_P bounds its coset's
    exact minimum from above (Eqs. (18)-(21)); on six syndromes at p = 0.25,
    the hardest noise of the workload."""
    L = O.Lattice(O.ROTATED, 11)
    p, eta = 0.25, 100.0
    w, wg = O.weights(p, O.noise(p, eta))
    beta = O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, 2000)
    rng = np.random.default_rng(111)
    for uid in range(6):
        _, syn = random_problem(L, p, eta, rng)
        out = L.decode(w, wg, syn, uid, 32, beta, 5, 6)
        exact = [_exact.coset_minimum_c(L.fq, L.fm, out["refs"][0] ^ L.logical(P), w) for P in range(4)]
        assert all(out["e_cls"][P] >= exact[P] for P in range(4))
        assert out["e_best"] >= min(exact)
