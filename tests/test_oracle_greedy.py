"""Pins for the oracle's greedy matching (Algs. 5-6, Eqs. (25)-(34)).

* syndrome consistency dR = S (Eq. (4)) for every mode and layout;
* the planar distance tables equal the paper's closed forms, Eqs. (26)-(30);
* the rotated tables equal an independent shortest-path computation;
* the matched pairs equal an independent implementation of the greedy rule
  (a different algorithm: repeated mutual-best-pair elimination, which gives
  the same matching as the sequential scan under a strict total order);
* the matching weight is bounded below by minimum-weight perfect matching;
* randomized tie breaking picks uniformly inside K_min (Eq. (34)).

The byte-exact tie order itself is a reading (the paper only asks for a
uniform pick), so it is the oracle's definition, not a paper pin.
"""
import itertools

import networkx as nx
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

LAYOUTS = [(O.ROTATED, d) for d in (3, 5, 7, 9, 11)] + [(O.PLANAR, d) for d in (3, 5, 7)]


def _syndromes(L, rng, n):
    out = []
    for i in range(n):
        if i % 2 == 0:
            out.append(rng.integers(0, 2, L.nstab).astype(np.uint8))
        else:
            p = rng.uniform(0.02, 0.3)
            e = np.where(rng.random(L.nq) < p, rng.integers(1, 4, L.nq), 0).astype(np.uint8)
            out.append(L.syndrome(e))
    return out


@pytest.mark.parametrize("layout,d", LAYOUTS)
def test_greedy_is_syndrome_consistent(layout, d):
    L = O.Lattice(layout, d)
    rng = np.random.default_rng(d)
    for p, eta in [(0.1, 10.0), (0.2, 1.0)]:
        _, wg = O.weights(p, O.noise(p, eta))
        for i, syn in enumerate(_syndromes(L, rng, 30)):
            for mode in (O.GREEDY_RANDOM, O.GREEDY_SAME, O.GREEDY_BOUNDARY):
                R = L.greedy(wg, syn, i, 3, 42, mode)
                assert np.array_equal(L.syndrome(R), syn)


@pytest.mark.parametrize("d", [3, 5, 7, 9])
def test_planar_distances_closed_form(d):
    """Eqs. (26)-(30) with unequal weights: interior distance
    W~z|dx| + W~x|dy|; white boundary W~x min(y, d-y); gray W~z min(x, d-x),
    in the paper's face coordinates (Sec. IV.B.1)."""
    L = O.Lattice(O.PLANAR, d)
    wg = np.array([70001, 130003], np.int32)  # W~x, W~z
    for g in (0, 1):
        dint, db, cf = L.tables(wg, g)
        xy = L.fxy[cf]
        if g == 0:   # white (i,j) at doubled (2i, 2j)
            ij = np.stack([xy[:, 0] // 2, xy[:, 1] // 2], 1)
            exp_db = wg[0] * np.minimum(ij[:, 1], d - ij[:, 1])
        else:        # gray (i,j) at doubled (2i+1, 2j-1)
            ij = np.stack([(xy[:, 0] - 1) // 2, (xy[:, 1] + 1) // 2], 1)
            exp_db = wg[1] * np.minimum(ij[:, 0], d - ij[:, 0])
        dx = np.abs(ij[:, None, 0] - ij[None, :, 0])
        dy = np.abs(ij[:, None, 1] - ij[None, :, 1])
        assert np.array_equal(dint, wg[1] * dx + wg[0] * dy)
        assert np.array_equal(db, exp_db)


def _graph_from_syndromes(L, wg, g):
    """Decoding graph of colour g built from single-component syndromes."""
    G = nx.Graph()
    faces = [f for f in range(L.nstab) if L.fcolour[f] == g]
    G.add_nodes_from(faces)
    G.add_node("B")
    for q in range(L.nq):
        for code, w in ((2, int(wg[0])), (1, int(wg[1]))):
            e = np.zeros(L.nq, np.uint8)
            e[q] = code
            hit = [f for f in np.where(L.syndrome(e))[0] if L.fcolour[f] == g]
            if len(hit) == 2:
                G.add_edge(hit[0], hit[1], weight=w)
            elif len(hit) == 1:
                old = G.get_edge_data(hit[0], "B")
                if old is None or old["weight"] > w:
                    G.add_edge(hit[0], "B", weight=w)
    return G, faces


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 3), (O.ROTATED, 7), (O.ROTATED, 11), (O.PLANAR, 5)])
def test_distances_match_shortest_paths(layout, d):
    L = O.Lattice(layout, d)
    wg = np.array([90001, 60013], np.int32)
    for g in (0, 1):
        dint, db, cf = L.tables(wg, g)
        G, faces = _graph_from_syndromes(L, wg, g)
        assert list(cf) == faces
        Gi = G.copy()
        Gi.remove_node("B")
        for a, fa in enumerate(faces):
            sp = nx.single_source_dijkstra_path_length(Gi, fa)
            assert [sp[fb] for fb in faces] == dint[a].tolist()
        spb = nx.single_source_dijkstra_path_length(G, "B")
        assert [spb[f] for f in faces] == db.tolist()
    if layout == O.ROTATED:
        # interior closed form on the rotated grid between cells (i,j):
        # W~z |di+dj|/2 + W~x |dj-di|/2 (diagonal Z steps, anti-diagonal X steps)
        for g in (0, 1):
            dint, _, cf = L.tables(wg, g)
            ij = L.fxy[cf]
            bulk = (ij[:, 0] >= 0) & (ij[:, 0] <= d - 2) & (ij[:, 1] >= 0) & (ij[:, 1] <= d - 2)
            di = ij[:, None, 0] - ij[None, :, 0]
            dj = ij[:, None, 1] - ij[None, :, 1]
            closed = wg[1] * np.abs(di + dj) // 2 + wg[0] * np.abs(dj - di) // 2
            sel = bulk[:, None] & bulk[None, :]
            assert np.array_equal(dint[sel], closed[sel])


def _independent_greedy(dint, db, defects, uid, rep, g, seed, randomized):
    """Mutual-best elimination: repeatedly match every pair that is the
    smallest remaining pair (by weight, key, id) for both of its ends."""
    nd = len(defects)
    na = nd + (nd & 1)

    def w(i, j):
        if j == nd:
            return int(db[defects[i]])
        return int(min(dint[defects[i], defects[j]], db[defects[i]] + db[defects[j]]))

    def key(i, j):
        pid = i * na + j
        return int(O.philox([uid, rep, 0x100 + g, pid], [seed & 0xFFFFFFFF, seed >> 32])[0]) if randomized else 0

    order = {}
    for i in range(na):
        for j in range(i + 1, na):
            order[(i, j)] = (w(i, j), key(i, j), i * na + j)
    free = set(range(na))
    pairs = set()
    while free:
        best = {}
        for (i, j), o in order.items():
            if i in free and j in free:
                for v in (i, j):
                    if v not in best or o < order[best[v]]:
                        best[v] = (i, j)
        for v, e in best.items():
            if e[0] == v and best[e[1]] == e:
                pairs.add(e)
        for e in list(pairs):
            free.discard(e[0])
            free.discard(e[1])
    return pairs


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 5), (O.ROTATED, 9), (O.PLANAR, 5)])
@pytest.mark.parametrize("mode", [O.GREEDY_RANDOM, O.GREEDY_SAME])
def test_matching_is_the_greedy_rule(layout, d, mode):
    L = O.Lattice(layout, d)
    p, eta = 0.15, 10.0
    _, wg = O.weights(p, O.noise(p, eta))
    rng = np.random.default_rng(100 + d)
    seed = 0x1234_5678_9ABC
    for uid, syn in enumerate(_syndromes(L, rng, 12)):
        for g in (0, 1):
            dint, db, cf = L.tables(wg, g)
            defects = [a for a, f in enumerate(cf) if syn[f]]
            got = L.greedy_pairs(wg, syn, uid, 5, seed, mode, g)
            ref = _independent_greedy(dint, db, defects, uid, 5, g, seed, mode == O.GREEDY_RANDOM)
            assert set(map(tuple, got.tolist())) == ref
            assert len(got) == (len(defects) + 1) // 2


def _chain_weight(L, wg, R, g):
    """Weight of the part of configuration R on the colour-g graph."""
    tot = 0
    for q in range(L.nq):
        for bit, w in ((2, int(wg[0])), (1, int(wg[1]))):
            if R[q] & bit:
                e = np.zeros(L.nq, np.uint8)
                e[q] = bit
                if L.fcolour[np.where(L.syndrome(e))[0][0]] == g:
                    tot += w
    return tot


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 5), (O.ROTATED, 7), (O.PLANAR, 5)])
def test_matching_weight_bounds(layout, d):
    """Minimum-weight perfect matching (Sec. IV.B.1) lower-bounds the weight of
    any syndrome-consistent chain, in particular the greedy one; the greedy
    chain weighs no more than the sum of its matched pair weights."""
    L = O.Lattice(layout, d)
    _, wg = O.weights(0.12, O.noise(0.12, 3.0))
    rng = np.random.default_rng(200 + d)
    for uid, syn in enumerate(_syndromes(L, rng, 10)):
        R = L.greedy(wg, syn, uid, 0, 9, O.GREEDY_RANDOM)
        for g in (0, 1):
            dint, db, cf = L.tables(wg, g)
            defects = [a for a, f in enumerate(cf) if syn[f]]
            nd = len(defects)
            H = nx.Graph()
            for i, j in itertools.combinations(range(nd), 2):
                H.add_edge(i, j, weight=int(min(dint[defects[i], defects[j]],
                                                db[defects[i]] + db[defects[j]])))
            for i in range(nd):
                H.add_edge(i, ("b", i), weight=int(db[defects[i]]))
            for i, j in itertools.combinations(range(nd), 2):
                H.add_edge(("b", i), ("b", j), weight=0)
            mwpm = sum(H.edges[e]["weight"] for e in nx.min_weight_matching(H)) if nd else 0
            pairs = L.greedy_pairs(wg, syn, uid, 0, 9, O.GREEDY_RANDOM, g)
            gw = sum(int(db[defects[i]]) if j == nd else
                     int(min(dint[defects[i], defects[j]], db[defects[i]] + db[defects[j]]))
                     for i, j in pairs)
            cw = _chain_weight(L, wg, R, g)
            assert mwpm <= cw <= gw


def test_modes():
    L = O.Lattice(O.ROTATED, 9)
    _, wg = O.weights(0.2, O.noise(0.2, 10.0))
    rng = np.random.default_rng(9)
    syn = _syndromes(L, rng, 2)[1]
    same = [L.greedy(wg, syn, 1, r, 5, O.GREEDY_SAME) for r in range(6)]
    assert all(np.array_equal(same[0], s) for s in same)
    rand = [L.greedy(wg, syn, 1, r, 5, O.GREEDY_RANDOM) for r in range(12)]
    assert len({s.tobytes() for s in rand}) > 1
    # Boundary mode: each defect goes to its nearest boundary (Sec. V.C)
    b = L.greedy(wg, syn, 1, 0, 5, O.GREEDY_BOUNDARY)
    for g in (0, 1):
        _, db, cf = L.tables(wg, g)
        assert _chain_weight(L, wg, b, g) <= sum(int(db[a]) for a, f in enumerate(cf) if syn[f])


def test_tie_breaking_is_uniform():
    """Eq. (34) / Alg. 6: the first pair is uniform over K_min.  Four isolated
    defects on a large lattice, arranged so that several pairs tie."""
    L = O.Lattice(O.ROTATED, 11)
    wg = np.array([100000, 100000], np.int32)
    dint, db, cf = L.tables(wg, 0)
    # pick defects of colour 0 forming a square: pairwise equal nearest distances
    cells = {tuple(L.fxy[f]): a for a, f in enumerate(cf)}
    quad = sorted([cells[(4, 4)], cells[(6, 4)], cells[(4, 6)], cells[(6, 6)]])
    syn = np.zeros(L.nstab, np.uint8)
    for a in quad:
        syn[cf[a]] = 1
    w = {}
    for i, j in itertools.combinations(range(4), 2):
        w[(i, j)] = int(min(dint[quad[i], quad[j]], db[quad[i]] + db[quad[j]]))
    wmin = min(w.values())
    kmin = [e for e, v in w.items() if v == wmin]
    assert len(kmin) >= 2
    counts = {e: 0 for e in kmin}
    n = 4000
    for r in range(n):
        first = tuple(L.greedy_pairs(wg, syn, 7, r, 31337, O.GREEDY_RANDOM, 0)[0].tolist())
        counts[first] += 1
    assert stats.chisquare(list(counts.values())).pvalue > 1e-3
