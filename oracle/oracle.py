"""ctypes wrapper around the plain-C oracle (xzzx_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the package smoke
check and by the CPU-baseline leg of the benchmark.  Nothing in the product
path imports it.  The wrapper only marshals arguments; all arithmetic is in
the C file, which cites the paper passage each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xzzx_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ROTATED, PLANAR = 0, 1
CONV_RATIO, CONV_PAPER = 0, 1
SCHED_LINEAR, SCHED_GEOMETRIC, SCHED_PAPER_LOG = 0, 1, 2
GREEDY_RANDOM, GREEDY_SAME, GREEDY_BOUNDARY = 0, 1, 2
ORDER_COLOUR, ORDER_RANDOM_SITE, ORDER_LADDER = 0, 1, 2   # colour sweeps; random-site steps (Alg. 3); replica exchange
RANK_DEFAULT, RANK_FACE_ID = 0, 1   # within-class rank orders (test hook: the reading of Alg. 3's visiting order)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math; strict IEEE double)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_lattice_new.restype = P
        L.or_lattice_new.argtypes = [C.c_int, C.c_int]
        L.or_lattice_free.argtypes = [P]
        L.or_lattice_nq.argtypes = [P]
        L.or_lattice_nstab.argtypes = [P]
        L.or_lattice_ncls.argtypes = [P, C.c_int]
        L.or_lattice_set_rank_order.argtypes = [P, C.c_int]
        L.or_lattice_export.argtypes = [P, i32p, u8p, i32p, i32p, i32p, i32p, u8p, u8p]
        L.or_noise.argtypes = [C.c_double, C.c_double, C.c_int, f64p]
        L.or_weights.argtypes = [C.c_double, f64p, i32p, i32p]
        L.or_energy.restype = C.c_int64
        L.or_energy.argtypes = [P, i32p, u8p]
        L.or_schedule.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, f64p]
        L.or_threshold.restype = C.c_uint32
        L.or_threshold.argtypes = [C.c_double, C.c_int64]
        L.or_syndrome.argtypes = [P, u8p, u8p]
        L.or_symp.argtypes = [P, u8p, u8p]
        L.or_class.argtypes = [P, u8p, u8p]
        L.or_class_mul.argtypes = [C.c_int, C.c_int]
        L.or_logical.argtypes = [P, C.c_int, u8p]
        L.or_build_tables.argtypes = [P, i32p]
        L.or_tables_export.argtypes = [P, i32p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_greedy.argtypes = [P, i32p, u8p, C.c_uint32, C.c_uint32, C.c_uint64, C.c_int, u8p]
        L.or_greedy_pairs.argtypes = [P, i32p, u8p, C.c_uint32, C.c_uint32, C.c_uint64, C.c_int,
                                      C.c_int, i32p]
        L.or_anneal_chain.argtypes = [P, i32p, f64p, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32,
                                      u8p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.or_anneal_chain_site.argtypes = L.or_anneal_chain.argtypes
        L.or_site_of.argtypes = [C.c_uint32, C.c_int]
        L.or_site_of.restype = C.c_uint32
        L.or_decode.argtypes = [P, i32p, i32p, u8p, C.c_uint32, C.c_int, f64p, C.c_int,
                                C.c_uint64, C.c_uint64, C.c_int,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double]
        L.or_reduce.argtypes = [C.c_int, i64p, i32p, i64p, C.c_void_p, C.c_void_p]
        L.or_swap_powers.argtypes = [C.c_double, C.c_void_p]
        L.or_swap_threshold.argtypes = [C.c_void_p, C.c_int64]
        L.or_swap_threshold.restype = C.c_uint32
        L.or_ladder_beta.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int]
        L.or_ladder_beta.restype = C.c_double
        L.or_anneal_ladder.argtypes = [P, i32p, C.c_double, C.c_double, C.c_int, C.c_int, C.c_uint64, C.c_uint32,
                                       C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def noise(p, eta, conv=CONV_RATIO):
    out = np.zeros(3, np.float64)
    rc = lib().or_noise(p, eta, conv, out)
    if rc:
        raise ValueError("or_noise: invalid arguments")
    return out


def weights(p, pxyz):
    w = np.zeros(4, np.int32)
    wg = np.zeros(2, np.int32)
    rc = lib().or_weights(p, np.ascontiguousarray(pxyz, np.float64), w, wg)
    if rc:
        raise ValueError("or_weights: invalid arguments")
    return w, wg


def schedule(kind, b0, b1, n):
    beta = np.zeros(max(n, 1), np.float64)
    rc = lib().or_schedule(kind, b0, b1, n, beta)
    if rc:
        raise ValueError("or_schedule: invalid arguments")
    return beta[:n]


def swap_powers(delta):
    out = np.zeros(32, np.uint64)
    lib().or_swap_powers(float(delta), _ptr(out))
    return out


def swap_threshold(R, n):
    R = np.ascontiguousarray(R, np.uint64)
    return int(lib().or_swap_threshold(_ptr(R), int(n)))


def ladder_beta(beta_lo, beta_hi, K, k):
    return float(lib().or_ladder_beta(float(beta_lo), float(beta_hi), int(K), int(k)))


def reduce(emin, cls):
    """Selection of Alg. 7 / Eq. (21) over chains with minima emin and cosets
    cls: (E_P[4], P*, best chain)."""
    emin = np.ascontiguousarray(emin, np.int64)
    cls = np.ascontiguousarray(cls, np.int32)
    e_cls = np.zeros(4, np.int64)
    ps = np.zeros(1, np.int32)
    bc = np.zeros(1, np.int32)
    if lib().or_reduce(len(emin), emin, cls, e_cls, _ptr(ps), _ptr(bc)):
        raise ValueError("or_reduce: class outside 0..3")
    return e_cls, int(ps[0]), int(bc[0])


def decode_by_chain(layout, d, w, wg, syn, uid, n_rep, beta, greedy_seed, anneal_seed, pool):
    """The oracle's decode of one syndrome (Alg. 7) assembled from its own
    steps, so that one large syndrome's chains run on the threads of `pool`
    (a concurrent.futures executor): the greedy reference of each replica
    (Alg. 6), its class relative to replica 0, every chain from R_r L_P
    (Algs. 2-3), then the selection of Eq. (21) (reduce).  Same fields as
    Lattice.decode(chains=True) without the final states and R_0 L_P*."""
    import threading
    local = threading.local()

    def lattice():
        if getattr(local, "lat", None) is None:
            local.lat = Lattice(layout, d)
        return local.lat

    uid = int(uid)
    refs = np.stack(list(pool.map(lambda r: lattice().greedy(wg, syn, uid, r, greedy_seed), range(n_rep))))
    lat = Lattice(layout, d)
    qcls = np.array([lat.cls(refs[r], refs[0]) for r in range(n_rep)], np.int32)

    def chain(c):
        L = lattice()
        return L.anneal_chain(w, beta, anneal_seed, uid, c, refs[c // 4] ^ L.logical(c % 4))

    res = list(pool.map(chain, range(4 * n_rep)))
    emin = np.array([r["emin"] for r in res], np.int64)
    cls = np.array([class_mul(qcls[c // 4], c % 4) for c in range(4 * n_rep)], np.int32)
    e_cls, ps, bc = reduce(emin, cls)
    return dict(refs=refs, qcls=qcls, chain_emin=emin, chain_stop=np.array([r["stop"] for r in res], np.int32),
                chain_e=np.array([r["e"] for r in res], np.int64), e_cls=e_cls, cls=ps, e_best=int(e_cls[ps]),
                best_chain=bc, recovery=res[bc]["snap"])


def class_mul(a, b):
    """Product of two logical classes (I=0, X=1, Y=2, Z=3)."""
    return int(lib().or_class_mul(int(a), int(b)))


def site_of(u, nstab):
    """Generator picked by a 32-bit site draw u among nstab (Alg. 3 step)."""
    return int(lib().or_site_of(int(u), int(nstab)))


def threshold(beta, dE):
    return int(lib().or_threshold(float(beta), int(dE)))


class Lattice:
    """Handle on the oracle's lattice (layout, distance d)."""

    def __init__(self, layout, d):
        self.h = lib().or_lattice_new(layout, d)
        if not self.h:
            raise ValueError(f"invalid lattice layout={layout} d={d}")
        self.layout, self.d = layout, d
        self.nq = lib().or_lattice_nq(self.h)
        self.nstab = lib().or_lattice_nstab(self.h)
        self.ncls = [lib().or_lattice_ncls(self.h, k) for k in range(4)]
        ns, nq = self.nstab, self.nq
        self.fq = np.zeros((ns, 4), np.int32)
        self.fm = np.zeros((ns, 4), np.uint8)
        self.fxy = np.zeros((ns, 2), np.int32)
        self.fclass = np.zeros(ns, np.int32)
        self.fcolour = np.zeros(ns, np.int32)
        self.frank = np.zeros(ns, np.int32)
        self.lx = np.zeros(nq, np.uint8)
        self.lz = np.zeros(nq, np.uint8)
        lib().or_lattice_export(self.h, self.fq, self.fm, self.fxy, self.fclass, self.fcolour,
                                self.frank, self.lx, self.lz)

    def set_rank_order(self, order):
        """Test hook: RANK_DEFAULT (the oracle's reading) or RANK_FACE_ID (the
        alternative reading, face-id order on both layouts)."""
        if lib().or_lattice_set_rank_order(self.h, int(order)):
            raise ValueError(f"unknown rank order {order}")
        lib().or_lattice_export(self.h, self.fq, self.fm, self.fxy, self.fclass, self.fcolour,
                                self.frank, self.lx, self.lz)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.or_lattice_free(h)
            self.h = None

    def energy(self, w, cfg):
        return int(lib().or_energy(self.h, np.ascontiguousarray(w, np.int32),
                                   np.ascontiguousarray(cfg, np.uint8)))

    def syndrome(self, cfg):
        cfg = np.ascontiguousarray(cfg, np.uint8)
        if cfg.ndim == 2:
            return np.stack([self.syndrome(c) for c in cfg])
        s = np.zeros(self.nstab, np.uint8)
        lib().or_syndrome(self.h, cfg, s)
        return s

    def symp(self, a, b):
        return int(lib().or_symp(self.h, np.ascontiguousarray(a, np.uint8),
                                 np.ascontiguousarray(b, np.uint8)))

    def cls(self, a, b):
        return int(lib().or_class(self.h, np.ascontiguousarray(a, np.uint8),
                                  np.ascontiguousarray(b, np.uint8)))

    def logical(self, P):
        out = np.zeros(self.nq, np.uint8)
        lib().or_logical(self.h, P, out)
        return out

    def tables(self, wg, g):
        n = sum(1 for c in self.fcolour if c == g)
        dint = np.zeros((n, n), np.int64)
        db = np.zeros(n, np.int64)
        cf = np.zeros(n, np.int32)
        rc = lib().or_tables_export(self.h, np.ascontiguousarray(wg, np.int32), g,
                                    _ptr(dint), _ptr(db), _ptr(cf))
        if rc < 0:
            raise ValueError("or_tables_export failed")
        return dint, db, cf

    def greedy(self, wg, syn, uid, rep, seed, mode=GREEDY_RANDOM):
        out = np.zeros(self.nq, np.uint8)
        rc = lib().or_greedy(self.h, np.ascontiguousarray(wg, np.int32),
                             np.ascontiguousarray(syn, np.uint8), uid, rep, seed, mode, out)
        if rc:
            raise RuntimeError(f"or_greedy rc={rc}")
        return out

    def greedy_pairs(self, wg, syn, uid, rep, seed, mode, g):
        pairs = np.zeros((self.nstab + 2, 2), np.int32)
        n = lib().or_greedy_pairs(self.h, np.ascontiguousarray(wg, np.int32),
                                  np.ascontiguousarray(syn, np.uint8), uid, rep, seed, mode, g, pairs)
        if n < 0:
            raise RuntimeError(f"or_greedy_pairs rc={n}")
        return pairs[:n]

    def anneal_chain(self, w, beta, seed, uid, chain, init, check=False, want_snap=True, order=ORDER_COLOUR):
        cfg = np.array(init, np.uint8, copy=True)
        e = np.zeros(1, np.int64)
        emin = np.zeros(1, np.int64)
        stop = np.zeros(1, np.int32)
        snap = np.zeros(self.nq, np.uint8) if want_snap else None
        beta = np.ascontiguousarray(beta, np.float64)
        fn = lib().or_anneal_chain_site if order == ORDER_RANDOM_SITE else lib().or_anneal_chain
        rc = fn(self.h, np.ascontiguousarray(w, np.int32), beta, len(beta),
                                   seed, uid, chain, cfg, _ptr(e), _ptr(emin), _ptr(stop),
                                   _ptr(snap), 1 if check else 0)
        if rc:
            raise RuntimeError(f"or_anneal_chain rc={rc}")
        return dict(final=cfg, e=int(e[0]), emin=int(emin[0]), stop=int(stop[0]), snap=snap)

    def anneal_ladder(self, w, beta_lo, beta_hi, K, n_sweeps, seed, uid, ladder, chain_ids, init, want_snap=True):
        """One ladder of K chains (replica exchange), all started from init [K][nq]."""
        cfg = np.array(init, np.uint8, copy=True).reshape(K, self.nq)
        e = np.zeros(K, np.int64)
        emin = np.zeros(K, np.int64)
        stop = np.zeros(K, np.int32)
        level = np.zeros(K, np.int32)
        snap = np.zeros((K, self.nq), np.uint8) if want_snap else None
        ids = np.ascontiguousarray(chain_ids, np.uint32)
        rc = lib().or_anneal_ladder(self.h, np.ascontiguousarray(w, np.int32), float(beta_lo), float(beta_hi), K,
                                    n_sweeps, seed, uid, ladder, _ptr(ids), _ptr(cfg), _ptr(e), _ptr(emin),
                                    _ptr(stop), _ptr(snap), _ptr(level))
        if rc:
            raise RuntimeError(f"or_anneal_ladder rc={rc}")
        return dict(final=cfg, e=e, emin=emin, stop=stop, snap=snap, level=level)

    def decode(self, w, wg, syn, uid, n_rep, beta, greedy_seed, anneal_seed,
               greedy_mode=GREEDY_RANDOM, check=False, chains=False, order=ORDER_COLOUR, ladder=(1, 1.0, 1.0)):
        """order ORDER_LADDER: replicas come in ladders of K = ladder[0] consecutive
        replicas sharing one greedy reference, at fixed levels from ladder[1] to
        ladder[2] (beta is then ignored except for its length, the sweep count)."""
        nq = self.nq
        nc = 4 * n_rep
        e_best = np.zeros(1, np.int64)
        cls_best = np.zeros(1, np.int32)
        e_cls = np.zeros(4, np.int64)
        rec = np.zeros(nq, np.uint8)
        prec = np.zeros(nq, np.uint8)
        best_chain = np.zeros(1, np.int32)
        refs = np.zeros((n_rep, nq), np.uint8)
        qcls = np.zeros(n_rep, np.int32)
        cemin = np.zeros(nc, np.int64) if chains else None
        cstop = np.zeros(nc, np.int32) if chains else None
        ce = np.zeros(nc, np.int64) if chains else None
        cfin = np.zeros((nc, nq), np.uint8) if chains else None
        beta = np.ascontiguousarray(beta, np.float64)
        rc = lib().or_decode(self.h, np.ascontiguousarray(w, np.int32),
                             np.ascontiguousarray(wg, np.int32),
                             np.ascontiguousarray(syn, np.uint8), uid, n_rep, beta, len(beta),
                             greedy_seed, anneal_seed, greedy_mode,
                             _ptr(e_best), _ptr(cls_best), _ptr(e_cls), _ptr(rec), _ptr(prec),
                             _ptr(best_chain), _ptr(refs), _ptr(qcls), _ptr(cemin), _ptr(cstop),
                             _ptr(ce), _ptr(cfin), 1 if check else 0, order, int(ladder[0]),
                             float(ladder[1]), float(ladder[2]))
        if rc:
            raise RuntimeError(f"or_decode rc={rc}")
        out = dict(e_best=int(e_best[0]), cls=int(cls_best[0]), e_cls=e_cls, recovery=rec,
                   paper_recovery=prec, best_chain=int(best_chain[0]), refs=refs, qcls=qcls)
        if chains:
            out.update(chain_emin=cemin, chain_stop=cstop, chain_e=ce, chain_final=cfin)
        return out
