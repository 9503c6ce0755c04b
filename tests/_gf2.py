"""Independent test-side mathematics over GF(2) for the XZZX code.

Nothing here calls the oracle's arithmetic: generators are read from the
lattice tables (positions and Pauli types only) and every quantity is
recomputed from first principles (symplectic algebra, exhaustive
enumeration), so these routines can pin the oracle.
"""
import numpy as np

X_BIT, Z_BIT = 2, 1


def generator_matrix(fq, fm, nq):
    """Generators as Pauli-code rows [nstab][nq] (I=0, Z=1, X=2, Y=3)."""
    G = np.zeros((len(fq), nq), np.uint8)
    for f in range(len(fq)):
        for s in range(4):
            if fq[f, s] >= 0:
                G[f, fq[f, s]] = fm[f, s]
    return G


def to_symplectic(P):
    """Pauli codes -> binary symplectic vectors (x | z)."""
    P = np.asarray(P, np.uint8)
    x = (P >> 1) & 1
    z = P & 1
    return np.concatenate([x, z], axis=-1)


def symp_products(A, B):
    """Matrix of symplectic products between rows of A and rows of B (mod 2)."""
    a = to_symplectic(A).astype(np.int64)
    b = to_symplectic(B).astype(np.int64)
    n = a.shape[-1] // 2
    lam = np.concatenate([b[..., n:], b[..., :n]], axis=-1)
    return (a @ lam.T) % 2


def gf2_rank(M):
    M = (np.asarray(M, np.uint8) & 1).copy()
    r = 0
    rows, cols = M.shape
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if M[i, c]:
                piv = i
                break
        if piv is None:
            continue
        M[[r, piv]] = M[[piv, r]]
        for i in range(rows):
            if i != r and M[i, c]:
                M[i] ^= M[r]
        r += 1
        if r == rows:
            break
    return r


def pack(cfg):
    """Pauli codes (nq <= 32) -> uint64 with X bits low, Z bits high."""
    cfg = np.asarray(cfg, np.uint8)
    nq = cfg.shape[-1]
    assert nq <= 32
    xw = np.zeros(cfg.shape[:-1], np.uint64)
    zw = np.zeros(cfg.shape[:-1], np.uint64)
    for q in range(nq):
        xw |= ((cfg[..., q] >> 1) & 1).astype(np.uint64) << np.uint64(q)
        zw |= (cfg[..., q] & 1).astype(np.uint64) << np.uint64(q)
    return xw | (zw << np.uint64(32))


def packed_energy(words, w):
    """Energy sum_q w[code_q] of packed configurations, w indexed I,Z,X,Y."""
    words = np.asarray(words, np.uint64)
    x = words & np.uint64(0xFFFFFFFF)
    z = words >> np.uint64(32)
    nx = np.bitwise_count(x & ~z).astype(np.int64)
    nz = np.bitwise_count(z & ~x).astype(np.int64)
    ny = np.bitwise_count(x & z).astype(np.int64)
    return int(w[2]) * nx + int(w[1]) * nz + int(w[3]) * ny


def group_elements(G):
    """All 2^r products of the generator rows (packed)."""
    gens = pack(G)
    arr = np.zeros(1, np.uint64)
    for g in gens:
        arr = np.concatenate([arr, arr ^ g])
    return arr


def coset_minima(group, base_cfgs, w):
    """Exact min of the energy over {base * G : G in group} for each base."""
    out = []
    for b in base_cfgs:
        e = packed_energy(group ^ pack(b), w)
        out.append(int(e.min()))
    return out
