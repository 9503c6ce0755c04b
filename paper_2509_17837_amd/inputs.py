"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds only workload definitions and random sampling --
none of the decoder's arithmetic.

The workload is code-capacity Pauli noise (the paper's Sec. IV.A channel):
each qubit independently suffers X, Y or Z with probabilities (p_x, p_y, p_z).
"""
from __future__ import annotations

import numpy as np

# Pauli codes: I=0, Z=1, X=2, Y=3
CODE_X, CODE_Y, CODE_Z = 2, 3, 1
CODE_I = 0


def channel(p: float, eta: float, convention: int = 0):
    """(p_x, p_y, p_z) of the sampled channel.  convention 0: p_y = p eta/(eta+1),
    p_x = p_z = p/(2(eta+1)); convention 1: p_x:p_y:p_z = 1:eta:1."""
    if convention == 0:
        return (p / (2 * (eta + 1)), p * eta / (eta + 1), p / (2 * (eta + 1)))
    return (p / (eta + 2), p * eta / (eta + 2), p / (eta + 2))


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
    easy as 1, 2, 3", SC'11) of counters ctr = (c0, c1, c2, c3) under key
    (k0, k1): uint32 arrays of one shape (or scalars) -> four uint32 arrays.
    The input sampler's own writing of the published generator (ten rounds of
    two 32 x 32 -> 64 multiplies by 0xD2511F53 and 0xCD9E8D57, the key bumped
    by 0x9E3779B9 and 0xBB67AE85)."""
    m32 = np.uint64(0xFFFFFFFF)
    c0, c1, c2, c3 = (np.asarray(c, np.uint64) & m32 for c in ctr)
    k0, k1 = (np.uint64(int(k) & 0xFFFFFFFF) for k in key)
    for _ in range(10):
        p0 = np.uint64(0xD2511F53) * c0
        p1 = np.uint64(0xCD9E8D57) * c2
        c0, c1, c2, c3 = (p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & m32, (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & m32
        k0 = (k0 + np.uint64(0x9E3779B9)) & m32
        k1 = (k1 + np.uint64(0xBB67AE85)) & m32
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def sample_errors(n: int, nq: int, pxyz, seed: int, stream: int = 0, uid0: int = 0) -> np.ndarray:
    """n i.i.d. error configurations [n][nq] (uint8 Pauli codes).  Qubit q of
    sample i draws u = word 0 of Philox4x32-10 with key (seed, stream) and
    counter (uid0 + i, q, 0x200, 0); with c1 = floor(2^32 p_x),
    c2 = floor(2^32 (p_x + p_y)), c3 = floor(2^32 (p_x + p_y + p_z)) the code
    is X if u < c1, else Y if u < c2, else Z if u < c3, else I."""
    px, py, pz = (float(v) for v in pxyz)
    c1, c2, c3 = (min(int(np.floor(np.ldexp(v, 32))), 1 << 32) for v in (px, px + py, px + py + pz))
    out = np.zeros((n, nq), np.uint8)
    q = np.arange(nq, dtype=np.uint64)
    rows = max(1, (1 << 20) // max(nq, 1))   # about 10^6 draws per chunk
    for a in range(0, n, rows):
        b = min(n, a + rows)
        i = (np.arange(a, b, dtype=np.uint64) + np.uint64(uid0))[:, None]
        u = philox4x32_10((np.broadcast_to(i, (b - a, nq)), np.broadcast_to(q, (b - a, nq)), 0x200, 0),
                          (seed, stream))[0].astype(np.int64)
        blk = out[a:b]
        blk[u < c3] = CODE_Z
        blk[u < c2] = CODE_Y
        blk[u < c1] = CODE_X
    return out


def sample_uids(n: int, first: int = 0) -> np.ndarray:
    return np.arange(first, first + n, dtype=np.uint32)


# The measured workloads.  The first five use the rotated layout and the
# channel of convention 0; the last is the paper's own set-up (Sec. IV.B, Sec. V):
# planar layout, p_x:p_y:p_z = 1:eta:1, the log schedule of Eqs. 23-24 from
# 0.9 beta_N to beta_N with N_beta = 100, N_SA = 10 references per syndrome.
# Seeds: sample 1000+k, greedy 2000+k, anneal 3000+k for workload k.
WORKLOADS = {
    "d3_small": dict(d=[3], p=[0.15], eta=[10.0], n_syn=1000, n_rep=1, sweeps=200,
                     schedule=("linear", 0.1, 5.0)),
    "d11_bias100": dict(d=[11], p=[0.10, 0.15, 0.20, 0.25], eta=[100.0], n_syn=100000, n_rep=32,
                        sweeps=2000, schedule=("geometric", 0.05, 10.0)),
    "mixed_d5_21": dict(d=[5, 9, 13, 17, 21], p=[0.18], eta=[10.0], n_syn=20000, n_rep=64, sweeps=5000,
                        schedule=("geometric", 0.05, 10.0)),
    "serving_d7_25": dict(d=[7, 11, 15, 19, 25], p=[0.12], eta=[1.0, 10.0, 1000.0], n_syn=20000, n_rep=16,
                          sweeps=1000, schedule=("geometric", 0.05, 10.0),
                          rates=[1e3, 3e3, 1e4, 3e4, 1e5]),
    "d31_large": dict(d=[31], p=[0.20], eta=[10.0], n_syn=10000, n_rep=128, sweeps=10000,
                      schedule=("geometric", 0.02, 20.0)),
    "planar_paper_d9": dict(layout="planar", convention="paper", d=[9], p=[0.10, 0.15], eta=[1.0, 5.0, 10.0],
                            n_syn=100000, n_rep=10, sweeps=100, schedule=("paper_log", 0.9, 1.0)),
}
WORKLOAD_INDEX = {name: k for k, name in enumerate(WORKLOADS)}
SCHEDULE_KIND = {"linear": 0, "geometric": 1, "paper_log": 2}
LAYOUT_KIND = {"rotated": 0, "planar": 1}
CONVENTION_KIND = {"ratio": 0, "paper": 1}


def layout_of(wl) -> int:
    return LAYOUT_KIND[wl.get("layout", "rotated")]


def convention_of(wl) -> int:
    return CONVENTION_KIND[wl.get("convention", "ratio")]


def seeds(name: str):
    k = WORKLOAD_INDEX[name]
    return dict(sample=1000 + k, greedy=2000 + k, anneal=3000 + k)


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (s) of n requests of a Poisson process."""
    rng = np.random.default_rng([int(seed), 7])
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
