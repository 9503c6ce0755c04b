"""CPU checks of the HIP library's host side (no kernel launches): the C ABI
loads and exports every declared symbol, and its plan-level arithmetic
(lattices, noise, weights, schedules, classes) agrees with the oracle."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_17837_amd import _lib as X
from paper_2509_17837_amd import decoder as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(xzzx_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    decl = declared_symbols()
    assert "xzzx_decode" in decl and "xzzx_anneal" in decl
    L = X.lib()
    missing = [n for n in sorted(decl) if not hasattr(L, n)]
    assert not missing, missing
    assert L.xzzx_version() == 1


@pytest.mark.parametrize("layout,d", [(0, 3), (0, 5), (0, 11), (0, 21), (0, 31), (1, 3), (1, 7), (1, 15)])
def test_lattice_matches_oracle(layout, d):
    a = D.Lattice(layout, d)
    b = O.Lattice(layout, d)
    assert (a.nq, a.nstab) == (b.nq, b.nstab)
    t = a.tables()
    assert np.array_equal(t["fq"], b.fq)
    assert np.array_equal(t["fm"], b.fm)
    assert np.array_equal(t["fclass"], b.fclass)
    assert np.array_equal(t["fcolour"], b.fcolour)
    assert np.array_equal(t["frank"], b.frank)
    lx, lz = a.logicals()
    assert np.array_equal(lx, b.lx) and np.array_equal(lz, b.lz)


def test_invalid_lattices_rejected():
    for layout, d in [(0, 2), (0, 1), (0, 33), (2, 5), (1, 4)]:
        with pytest.raises(X.XzzxError) as e:
            D.Lattice(layout, d)
        assert e.value.rc == X.XZZX_EINVAL


@pytest.mark.parametrize("conv", [0, 1])
def test_noise_weights_match_oracle(conv):
    rng = np.random.default_rng(1)
    for _ in range(200):
        p = float(rng.uniform(1e-4, 0.49))
        eta = float(10 ** rng.uniform(-2, 4))
        a = D.noise(p, eta, conv)
        b = O.noise(p, eta, conv)
        assert a.tobytes() == b.tobytes()
        wa, ga = D.weights(p, a)
        wb, gb = O.weights(p, b)
        assert np.array_equal(wa, wb) and np.array_equal(ga, gb)
    with pytest.raises(X.XzzxError):
        D.noise(0.6, 1.0)
    with pytest.raises(X.XzzxError):
        D.noise(0.1, 0.0)


@pytest.mark.parametrize("kind,b0,b1", [(0, 0.1, 5.0), (1, 0.05, 10.0), (1, 0.02, 20.0), (2, 0.9, 1.0)])
def test_schedules_match_oracle(kind, b0, b1):
    for n in (0, 1, 2, 7, 200, 2000, 10000):
        a = D.schedule(kind, b0, b1, n)
        b = O.schedule(kind, b0, b1, n)
        assert a.tobytes() == b.tobytes()


def test_class_host_matches_oracle():
    for layout, d in [(0, 5), (1, 5)]:
        a = D.Lattice(layout, d)
        b = O.Lattice(layout, d)
        rng = np.random.default_rng(2)
        for _ in range(50):
            e = rng.integers(0, 4, a.nq).astype(np.uint8)
            base = rng.integers(0, 4, a.nq).astype(np.uint8)
            assert a.cls(base, base ^ e) == b.cls(base, base ^ e)
            P = int(rng.integers(0, 4))
            assert a.cls(base, base ^ b.logical(P)) == P


def test_energy_overflow_is_erange():
    """ERANGE when n_qubits * max(W) >= 2^31 (energies are int32 sums of the
    weights of Eq. (10)); checked before any device work, so it runs without
    a GPU.  One unit below the limit passes that check (and then needs a GPU
    for the plan's device tables)."""
    lat = D.Lattice(X.ROTATED, 31)
    assert lat.nq == 961
    at_limit = -(-(1 << 31) // lat.nq)            # least w with 961 w >= 2^31
    assert lat.nq * at_limit >= 1 << 31 > lat.nq * (at_limit - 1)
    for slot in (1, 2, 3):
        w = np.array([0, 1000, 1000, 1000], np.int32)
        w[slot] = at_limit
        with pytest.raises(X.XzzxError) as e:
            D.Plan(lat, w, np.array([500, 500], np.int32), np.zeros(0))
        assert e.value.rc == X.XZZX_ERANGE
    w = np.array([0, at_limit - 1, 1000, 1000], np.int32)
    try:
        D.Plan(lat, w, np.array([500, 500], np.int32), np.zeros(0))
    except X.XzzxError as e:
        assert e.rc != X.XZZX_ERANGE
