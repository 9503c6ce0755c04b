"""Exact minimum energy of a coset {C0 * prod_f G_f^(x_f)} by variable
elimination over the generator bits in face-id order (a frontier dynamic
program), written independently of the oracle for tests: each qubit's
weight is added once every generator touching it has been fixed, and a
generator leaves the frontier once no unfinished qubit depends on it.  Exact
for any lattice; fast while the frontier stays small (about d + 2 bits on
the rotated lattice in row-major order)."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DP_SRC = os.path.join(HERE, "_exact_dp.c")
DP_LIB = os.path.join(HERE, "_exact_dp.so")
_dp = None


def build_dp(force=False):
    """Compile the C form of the frontier program (tests/_exact_dp.c)."""
    if force or not os.path.exists(DP_LIB) or os.path.getmtime(DP_LIB) < os.path.getmtime(DP_SRC):
        tmp = DP_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, DP_SRC])
        os.replace(tmp, DP_LIB)
    return DP_LIB


def coset_minimum_c(fq, fm, c0, w):
    """The frontier program of coset_minimum in C (tests/_exact_dp.c)."""
    global _dp
    if _dp is None:
        build_dp()
        L = C.CDLL(DP_LIB)
        L.dp_coset_minimum.restype = C.c_int64
        L.dp_coset_minimum.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _dp = L
    fq = np.ascontiguousarray(fq, np.int32)
    fm = np.ascontiguousarray(fm, np.uint8)
    c0 = np.ascontiguousarray(c0, np.uint8)
    w = np.ascontiguousarray(w, np.int32)
    r = _dp.dp_coset_minimum(len(c0), len(fq), fq.ctypes.data, fm.ctypes.data, c0.ctypes.data, w.ctypes.data)
    if r < 0:
        raise RuntimeError(f"dp_coset_minimum failed ({r})")
    return int(r)


def coset_minimum(fq, fm, c0, w):
    fq = np.asarray(fq)
    fm = np.asarray(fm)
    c0 = np.asarray(c0, np.uint8)
    nstab, nq = fq.shape[0], c0.shape[0]
    touching = [[] for _ in range(nq)]            # (generator, Pauli code) pairs per qubit
    for f in range(nstab):
        for s in range(4):
            q = int(fq[f, s])
            if q >= 0:
                touching[q].append((f, int(fm[f, s])))
    last = [max((f for f, _ in t), default=-1) for t in touching]
    const = sum(int(w[c0[q]]) for q in range(nq) if last[q] < 0)
    done_at = [[] for _ in range(nstab)]
    for q in range(nq):
        if last[q] >= 0:
            done_at[last[q]].append(q)
    # a generator is needed until the last of its qubits is finished
    needed_until = [max(last[int(q)] for q in fq[f] if q >= 0) for f in range(nstab)]
    frontier = []                                  # generator ids, bit i of a state = frontier[i]
    states = {0: const}
    for g in range(nstab):
        frontier.append(g)
        pos = {f: i for i, f in enumerate(frontier)}
        new = {}
        for st, cost in states.items():
            for bit in (0, 1):
                s2 = st | (bit << pos[g])
                c = cost
                for q in done_at[g]:
                    code = int(c0[q])
                    for f, m in touching[q]:
                        if (s2 >> pos[f]) & 1:
                            code ^= m
                    c += int(w[code])
                if c < new.get(s2, 1 << 62):
                    new[s2] = c
        # drop generators no longer needed, merging states by their minimum
        keep = [f for f in frontier if needed_until[f] > g]
        if len(keep) < len(frontier):
            idx = [pos[f] for f in keep]
            merged = {}
            for st, cost in new.items():
                s2 = 0
                for i, j in enumerate(idx):
                    s2 |= ((st >> j) & 1) << i
                if cost < merged.get(s2, 1 << 62):
                    merged[s2] = cost
            new = merged
            frontier = keep
        states = new
    return min(states.values())
