"""Pins for the oracle's random numbers, noise model, weights, schedules and
acceptance thresholds (Eqs. (5)-(12), (22)-(24); Alg. 3)."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    """Published known-answer vectors of Philox4x32-10 (Salmon et al., SC'11)."""
    for ctr, key, out in _kat():
        assert O.philox(ctr, key).tolist() == out


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
    unsigned a, b, c, d, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &a, &b, &c, &d, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c | ((unsigned long long)d << 32);
        unsigned long long off = 4ull * ((unsigned long long)a | ((unsigned long long)b << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand():
    """Cross-check against an independent implementation by calling rocRAND's
    host-callable Philox4x32-10 engine (counter = (offset/4, subsequence))."""
    rng = np.random.default_rng(11)
    cases = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    cases[:, 1] >>= 2  # the engine takes 4*(ctr0 + 2^32 ctr1) as a 64-bit offset
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "probe.cpp")
        exe = os.path.join(td, "probe")
        with open(src, "w") as fh:
            fh.write(ROCRAND_PROBE)
        subprocess.check_call(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-o", exe, src],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        inp = "\n".join(" ".join(str(int(x)) for x in row) for row in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    got = [list(map(int, line.split())) for line in out.strip().splitlines()]
    for row, ref in zip(cases, got):
        assert O.philox(row[:4], row[4:6]).tolist() == ref


def test_noise_conventions():
    # ratio form (eta = p_Y/(p_X + p_Z)): p_Y = p eta/(eta+1), p_X = p_Z = p/(2(eta+1))
    px, py, pz = O.noise(0.15, 10.0, O.CONV_RATIO)
    assert math.isclose(px + py + pz, 0.15, rel_tol=1e-15)
    assert px == pz and math.isclose(py / px, 20.0, rel_tol=1e-14)
    # Sec. V.A: p_x:p_y:p_z = 1:eta:1; eta=1 is depolarizing p/3 each
    px, py, pz = O.noise(0.3, 1.0, O.CONV_PAPER)
    assert math.isclose(px, 0.1) and math.isclose(py, 0.1) and math.isclose(pz, 0.1)
    px, py, pz = O.noise(0.12, 5.0, O.CONV_PAPER)
    assert math.isclose(py / px, 5.0) and px == pz
    for bad in [(0.0, 1.0), (0.5, 1.0), (0.1, 0.0), (0.1, -1.0)]:
        with pytest.raises(ValueError):
            O.noise(*bad)


# Expected integer weights of the measured workloads: round(2^16 * -ln(p_P/(1-p)))
# with the ratio noise form (values tabulated with the workload definitions).
WEIGHT_TABLE = [
    # p, eta, W_X(=W_Z), W_Y, W~
    (0.15, 10.0, 316253, 119925, 116728),
    (0.10, 100.0, 491880, 144649, 144323),
    (0.15, 100.0, 461561, 114331, 114004),
    (0.20, 100.0, 438735, 91504, 91177),
    (0.25, 100.0, 419881, 72651, 72324),
    (0.18, 10.0, 301950, 105622, 102424),
    (0.12, 1.0, 221428, 176002, 149429),
    (0.12, 10.0, 333150, 136822, 133625),
    (0.12, 1000.0, 628774, 130641, 130609),
    (0.20, 10.0, 293427, 97098, 93901),
]


@pytest.mark.parametrize("p,eta,wx,wy,wt", WEIGHT_TABLE)
def test_weights_table(p, eta, wx, wy, wt):
    w, wg = O.weights(p, O.noise(p, eta))
    assert w.tolist() == [0, wx, wx, wy]
    assert wg.tolist() == [wt, wt]


def test_weights_are_nishimori_scaled_alpha():
    """Eqs. (9), (12): W_mu / 2^16 = beta_N * alpha_mu = -ln(p_mu/(1-p))."""
    for p, eta, conv in [(0.07, 3.0, 0), (0.2, 0.5, 1), (0.01, 30.0, 1)]:
        pxyz = O.noise(p, eta, conv)
        w, wg = O.weights(p, pxyz)
        beta_n = -math.log(p / (1 - p))
        for idx, pm in ((2, pxyz[0]), (3, pxyz[1]), (1, pxyz[2])):
            alpha = math.log(pm / (1 - p)) / math.log(p / (1 - p))
            assert abs(w[idx] / 65536.0 - beta_n * alpha) <= 0.5 / 65536 + 1e-12
        assert abs(wg[0] / 65536.0 + math.log((pxyz[0] + pxyz[1]) / (1 - p))) <= 0.5 / 65536 + 1e-12
        assert abs(wg[1] / 65536.0 + math.log((pxyz[2] + pxyz[1]) / (1 - p))) <= 0.5 / 65536 + 1e-12


def test_schedules():
    lin = O.schedule(O.SCHED_LINEAR, 0.1, 5.0, 200)
    assert lin[0] == 0.1 and lin[-1] == 5.0 and np.all(np.diff(lin) > 0)
    assert np.allclose(np.diff(lin), (5.0 - 0.1) / 199, rtol=1e-9)
    geo = O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, 2000)
    assert geo[0] == 0.05 and math.isclose(geo[-1], 10.0, rel_tol=1e-14)
    r = geo[1:] / geo[:-1]
    assert np.allclose(r, (10.0 / 0.05) ** (1 / 1999), rtol=1e-12)
    # Eqs. (23)-(24): beta_1 = beta_init, beta_{N} = beta_final, log spacing
    pl = O.schedule(O.SCHED_PAPER_LOG, 0.9, 1.0, 100)
    assert pl[0] == 0.9 and math.isclose(pl[-1], 1.0, rel_tol=1e-14)
    gamma = (1.0 / 0.9 - 1.0) / math.log(100)
    assert np.allclose(pl, 0.9 * (1 + gamma * np.log(np.arange(1, 101))), rtol=1e-14)
    # N_beta in {0,1}: gamma = 0
    assert O.schedule(O.SCHED_PAPER_LOG, 0.9, 1.0, 1).tolist() == [0.9]
    assert len(O.schedule(O.SCHED_PAPER_LOG, 0.9, 1.0, 0)) == 0
    assert O.schedule(O.SCHED_LINEAR, 0.3, 7.0, 1).tolist() == [0.3]


def test_threshold_rule():
    """Alg. 3: accept iff r < min{1, exp(-beta dE)}, r = u/2^32."""
    two32 = 2.0 ** 32
    assert O.threshold(1.0, 0) == 0xFFFFFFFF and O.threshold(1.0, -5) == 0xFFFFFFFF
    assert O.threshold(0.0, 123456) == 0xFFFFFFFF          # beta = 0: accept all
    assert O.threshold(10.0, 65536 * 100) == 0              # exp(-1000) underflows
    rng = np.random.default_rng(5)
    for _ in range(2000):
        beta = float(rng.uniform(0.01, 20.0))
        dE = int(rng.integers(1, 3_000_000))
        T = O.threshold(beta, dE)
        x = math.exp(-(beta * dE) / 65536.0)
        # T = ceil(2^32 x): the integer rule u < T is exactly u / 2^32 < x
        assert T - 1 < two32 * x <= T or (T == 0xFFFFFFFF and two32 * x > T - 1)
        if 0 < T < 0xFFFFFFFF:
            assert (T - 1) / two32 < x and not (T / two32 < x)
    # monotone in dE and in beta
    ts = [O.threshold(0.7, d) for d in range(1, 400000, 997)]
    assert all(a >= b for a, b in zip(ts, ts[1:]))
