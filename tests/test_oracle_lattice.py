"""Pins for the oracle's code model (Sec. II, Eq. (1), Eqs. (2)-(4), Sec. III).

Each property is fixed by the paper or by stabilizer-code algebra and is
recomputed here independently of the oracle (tests/_gf2.py).
"""
import itertools

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

from oracle import oracle as O
from tests import _gf2

CASES = [(O.ROTATED, d) for d in (3, 5, 7, 9, 11)] + [(O.PLANAR, d) for d in (3, 5, 7, 9)]


@pytest.mark.parametrize("layout,d", CASES)
def test_counts(layout, d):
    L = O.Lattice(layout, d)
    if layout == O.PLANAR:
        # Sec. II: N_q = d^2 + (d-1)^2 and N_stab = 2d(d-1)
        assert L.nq == d * d + (d - 1) * (d - 1)
        assert L.nstab == 2 * d * (d - 1)
        # Sec. IV.B.1: white faces (i,j), i=1..d, j=1..d-1 ; gray i=1..d-1, j=1..d
        assert (L.fcolour == 0).sum() == d * (d - 1)
        assert (L.fcolour == 1).sum() == (d - 1) * d
    else:
        assert L.nq == d * d and L.nstab == d * d - 1


@pytest.mark.parametrize("layout,d", CASES)
def test_generators_are_xzzx(layout, d):
    """Eq. (1): X on left/right, Z on up/down; four-body in the bulk and fewer
    at the boundaries (three-body on the planar layout)."""
    L = O.Lattice(layout, d)
    weights = (L.fq >= 0).sum(1)
    for f in range(L.nstab):
        present = L.fq[f] >= 0
        assert list(L.fm[f][present]) == [m for m, p in zip([2, 1, 1, 2], present) if p]
    assert weights.max() == 4
    assert (weights == 4).sum() == (L.nstab - 4 * ((d - 1) // 2) if layout == O.ROTATED
                                    else L.nstab - 4 * (d - 1))
    expect_boundary_weight = 2 if layout == O.ROTATED else 3
    assert set(weights[weights < 4]) == {expect_boundary_weight}


@pytest.mark.parametrize("layout,d", CASES)
def test_stabilizer_algebra(layout, d):
    L = O.Lattice(layout, d)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    # all generators commute
    assert not _gf2.symp_products(G, G).any()
    # independent: rank = N_stab (so every syndrome pattern is reachable)
    assert _gf2.gf2_rank(_gf2.to_symplectic(G)) == L.nstab
    # logicals commute with the group, anticommute with each other, and are
    # not in the group
    Ls = np.stack([L.lx, L.lz])
    assert not _gf2.symp_products(G, Ls).any()
    assert _gf2.symp_products(L.lx[None], L.lz[None])[0, 0] == 1
    full = _gf2.to_symplectic(np.concatenate([G, Ls]))
    assert _gf2.gf2_rank(full) == L.nstab + 2
    # L_X runs between the top and bottom boundaries and L_Z between the
    # left and right ones, each of weight d (Sec. II, code distance d)
    assert (L.lx > 0).sum() == d and (L.lz > 0).sum() == d


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 3), (O.PLANAR, 3), (O.ROTATED, 5)])
def test_code_distance(layout, d):
    """Sec. II: the code distance is d -- no nontrivial logical operator has
    weight below d (exhaustive over all Pauli operators of weight < d), and
    L_X, L_Z have weight d."""
    L = O.Lattice(layout, d)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    Gs = _gf2.to_symplectic(G)
    r = _gf2.gf2_rank(Gs)
    for wt in range(1, d):
        subsets = np.array(list(itertools.combinations(range(L.nq), wt)), np.int64)
        paulis = np.array(list(itertools.product((1, 2, 3), repeat=wt)), np.uint8)
        for chunk in np.array_split(subsets, max(1, len(subsets) // 2000)):
            cand = np.zeros((len(chunk), len(paulis), L.nq), np.uint8)
            rows = np.arange(len(chunk))[:, None, None]
            cols = np.arange(len(paulis))[None, :, None]
            cand[rows, cols, chunk[:, None, :]] = paulis[None, :, :]
            cand = cand.reshape(-1, L.nq)
            comm = ~_gf2.symp_products(cand, G).any(axis=1)
            for P in cand[comm]:
                # commutes with the whole group: must itself be a stabilizer
                assert _gf2.gf2_rank(np.concatenate([Gs, _gf2.to_symplectic(P[None])])) == r
    assert (L.lx > 0).sum() == d and (L.lz > 0).sum() == d


@pytest.mark.parametrize("layout,d", CASES)
def test_colour_classes(layout, d):
    """Generators of one class act on disjoint qubits, and the four classes
    have equal size N_stab/4 -- the condition for updating a class at once."""
    L = O.Lattice(layout, d)
    for k in range(4):
        faces = np.where(L.fclass == k)[0]
        assert len(faces) == L.nstab // 4 == L.ncls[k]
        qs = L.fq[faces][L.fq[faces] >= 0]
        assert len(qs) == len(set(qs.tolist()))
        assert sorted(L.frank[faces].tolist()) == list(range(len(faces)))


@pytest.mark.parametrize("layout,d", CASES)
def test_decoding_graphs(layout, d):
    """Sec. III: a single X or Z component flips one or two faces, all of one
    colour; X and Z components of one qubit live on different colours."""
    L = O.Lattice(layout, d)
    for q in range(L.nq):
        cols = []
        for code in (1, 2):
            e = np.zeros(L.nq, np.uint8)
            e[q] = code
            s = L.syndrome(e)
            hit = np.where(s)[0]
            assert 1 <= len(hit) <= 2
            assert len(set(L.fcolour[hit].tolist())) == 1
            cols.append(L.fcolour[hit[0]])
        assert cols[0] != cols[1]


@pytest.mark.parametrize("layout,d", CASES[:3] + CASES[5:7])
def test_syndrome_is_symplectic_product(layout, d):
    """Eq. (2): s_f = 1 iff C anticommutes with G_f; the syndrome is linear."""
    L = O.Lattice(layout, d)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    rng = np.random.default_rng(7)
    for _ in range(20):
        a = rng.integers(0, 4, L.nq).astype(np.uint8)
        b = rng.integers(0, 4, L.nq).astype(np.uint8)
        sa = L.syndrome(a)
        assert np.array_equal(sa, _gf2.symp_products(G, a[None])[:, 0].astype(np.uint8))
        assert np.array_equal(L.syndrome(a ^ b), sa ^ L.syndrome(b))


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 3), (O.ROTATED, 7), (O.PLANAR, 5)])
def test_class_function(layout, d):
    """Logical class via commutation with L_X and L_Z (Alg. 7): exact on the
    representatives, invariant under stabilizers, -1 off the syndrome-free set."""
    L = O.Lattice(layout, d)
    G = _gf2.generator_matrix(L.fq, L.fm, L.nq)
    zero = np.zeros(L.nq, np.uint8)
    assert L.cls(L.lx, zero) == 1 and L.cls(L.lz, zero) == 3
    assert L.cls(L.lx ^ L.lz, zero) == 2 and L.cls(zero, zero) == 0
    rng = np.random.default_rng(3)
    for P in range(4):
        rep = L.logical(P)
        for _ in range(5):
            sel = rng.integers(0, 2, L.nstab).astype(bool)
            stab = np.bitwise_xor.reduce(G[sel], axis=0) if sel.any() else zero
            assert L.cls(rep ^ stab, zero) == P
    e = zero.copy()
    e[0] = 2
    assert L.cls(e, zero) == -1
    # Pauli product table of class indices I, X, Y, Z
    table = [[0, 1, 2, 3], [1, 0, 3, 2], [2, 3, 0, 1], [3, 2, 1, 0]]
    for a in range(4):
        for b in range(4):
            assert O.lib().or_class_mul(a, b) == table[a][b]


@pytest.mark.parametrize("layout,d", [(O.ROTATED, 5), (O.ROTATED, 9), (O.PLANAR, 3), (O.PLANAR, 7), (O.PLANAR, 9)])
def test_within_class_rank_order(layout, d):
    """The rank of a generator in its colour class (it names the random word
    the generator draws): face-id order on the rotated lattice; on the planar
    lattice row-major over ((x + y)/2, (x - y)/2), the generator's 2 x 2 block
    in the lattice turned by 45 degrees, where consecutive ranks of a class
    share a pair of rows."""
    L = O.Lattice(layout, d)
    for k in range(4):
        faces = np.where(L.fclass == k)[0]
        ordered = faces[np.argsort(L.frank[faces])]
        if layout == O.ROTATED:
            assert ordered.tolist() == sorted(faces.tolist())
        else:
            x, y = L.fxy[ordered, 0], L.fxy[ordered, 1]
            keys = list(zip(((x + y) // 2).tolist(), ((x - y) // 2).tolist()))
            assert keys == sorted(keys) and len(set(keys)) == len(keys)
            # a class's blocks of one row pair are disjoint and consecutive
            rows = [a for a, _ in keys]
            assert rows == sorted(rows)


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(layout=st.sampled_from([O.ROTATED, O.PLANAR]), d=st.sampled_from([3, 5, 7]),
       seed=st.integers(0, 2**32 - 1), p=st.floats(0.02, 0.3), eta=st.floats(0.5, 200.0))
def test_random_problems_keep_the_invariants(layout, d, seed, p, eta):
    """Property test over random lattices, channels and seeds: a short
    annealing chain keeps its syndrome, coset and incremental energy after
    every sweep (the oracle's check mode), its snapshot has energy E_min, and
    the greedy reference has the sampled syndrome."""
    L = O.Lattice(layout, d)
    pxyz = O.noise(p, eta)
    w, wg = O.weights(p, pxyz)
    rng = np.random.default_rng(seed)
    u = rng.random(L.nq)
    err = np.zeros(L.nq, np.uint8)
    err[u < pxyz[0] + pxyz[1] + pxyz[2]] = 1
    err[u < pxyz[0] + pxyz[1]] = 3
    err[u < pxyz[0]] = 2
    syn = L.syndrome(err)
    ref = L.greedy(wg, syn, seed & 0xFFFF, 1, seed)
    assert np.array_equal(L.syndrome(ref), syn)
    beta = O.schedule(O.SCHED_GEOMETRIC, 0.1, 5.0, 12)
    r = L.anneal_chain(w, beta, seed, seed & 0xFFFF, 3, ref, check=True)
    assert L.energy(w, r["snap"]) == r["emin"] <= r["e"]
    assert L.cls(r["final"], ref) == 0
