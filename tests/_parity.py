"""Shared helpers of the GPU parity tests: build a seeded problem, run the
oracle (CPU, threaded over syndromes) and the HIP path (through the C ABI),
and compare element by element."""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import oracle as O
from paper_2509_17837_amd import inputs

_POOL = None


def pool():
    global _POOL
    if _POOL is None:
        _POOL = ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4))
    return _POOL


class Problem:
    def __init__(self, layout, d, p, eta, n_syn, n_rep, n_sweeps, sched=("geometric", 0.05, 10.0),
                 seed=11, conv=0, uid0=0, beta=None):
        self.layout, self.d, self.p, self.eta, self.conv = layout, d, p, eta, conv
        self.n_syn, self.n_rep, self.n_sweeps = n_syn, n_rep, n_sweeps
        self.olat = O.Lattice(layout, d)
        self.pxyz = O.noise(p, eta, conv)
        self.w, self.wg = O.weights(p, self.pxyz)
        kind = inputs.SCHEDULE_KIND[sched[0]]
        self.sched = (kind, sched[1], sched[2])
        self.custom_beta = None if beta is None else np.asarray(beta, np.float64)
        self.beta = O.schedule(kind, sched[1], sched[2], n_sweeps) if beta is None else self.custom_beta
        self.errors = inputs.sample_errors(n_syn, self.olat.nq, inputs.channel(p, eta, conv), seed, stream=d)
        self.syn = np.stack([self.olat.syndrome(e) for e in self.errors]) if n_syn else \
            np.zeros((0, self.olat.nstab), np.uint8)
        self.uid = inputs.sample_uids(n_syn, uid0)
        self.greedy_seed = 0x5EED_0000 + seed
        self.anneal_seed = 0xA11E_0000_0000 + seed

    def oracle_decode(self, idx=None, mode=O.GREEDY_RANDOM, chains=True, order=O.ORDER_COLOUR, ladder=(1, 1.0, 1.0)):
        idx = range(self.n_syn) if idx is None else idx

        def one(i):
            lat = O.Lattice(self.layout, self.d)  # per-thread handle (greedy tables are cached per handle)
            return lat.decode(self.w, self.wg, self.syn[i], int(self.uid[i]), self.n_rep, self.beta,
                              self.greedy_seed, self.anneal_seed, mode, chains=chains, order=order, ladder=ladder)

        return list(pool().map(one, list(idx)))

    def oracle_chain(self, ref, qcls_unused, i, c):
        """One chain of syndrome i from reference `ref` (the replica's R_r)."""
        lat = O.Lattice(self.layout, self.d)
        P = c % 4
        init = ref ^ lat.logical(P)
        return lat.anneal_chain(self.w, self.beta, self.anneal_seed, int(self.uid[i]), c, init)

    def oracle_greedy(self, i, r, mode=O.GREEDY_RANDOM):
        lat = O.Lattice(self.layout, self.d)
        return lat.greedy(self.wg, self.syn[i], int(self.uid[i]), r, self.greedy_seed, mode)


def oracle_decode_by_chain(layout, d, w, wg, syn, uid, n_rep, beta, greedy_seed, anneal_seed):
    """oracle.decode_by_chain on the shared host thread pool."""
    return O.decode_by_chain(layout, d, w, wg, syn, uid, n_rep, beta, greedy_seed, anneal_seed, pool())


def gpu_plan(prob, lanes=None):
    from paper_2509_17837_amd import decoder as D
    lat = D.Lattice(prob.layout, prob.d)
    w, wg = D.weights(prob.p, D.noise(prob.p, prob.eta, prob.conv))
    assert np.array_equal(w, prob.w) and np.array_equal(wg, prob.wg)
    beta = D.schedule(*prob.sched, prob.n_sweeps) if prob.custom_beta is None else prob.custom_beta
    plan = D.Plan(lat, w, wg, beta)
    if lanes is not None:
        plan.set_lanes(lanes)
    return plan


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def compare_decode(prob, out, ref, check_chains=True):
    """Element-wise comparison of one group's GPU outputs with oracle results."""
    e_best = out.e_best.cpu().numpy()
    cls = out.cls.cpu().numpy()
    rec = out.recovery.cpu().numpy()
    for i, r in enumerate(ref):
        tag = f"syndrome {i} (uid {prob.uid[i]})"
        if out.refs is not None:
            assert np.array_equal(out.refs[i].cpu().numpy(), r["refs"]), tag + " refs"
        if out.qcls is not None:
            assert np.array_equal(out.qcls[i].cpu().numpy(), r["qcls"]), tag + " qcls"
        if check_chains and out.chain_emin is not None:
            assert np.array_equal(out.chain_emin[i].cpu().numpy(), r["chain_emin"]), tag + " chain E_min"
            assert np.array_equal(out.chain_stop[i].cpu().numpy(), r["chain_stop"]), tag + " chain stop"
            assert np.array_equal(out.chain_e[i].cpu().numpy(), r["chain_e"]), tag + " chain E"
        if check_chains and out.chain_final is not None:
            assert np.array_equal(out.chain_final[i].cpu().numpy(), r["chain_final"]), tag + " final states"
        assert e_best[i] == r["e_best"], tag + " E_best"
        assert cls[i] == r["cls"], tag + " class"
        if out.e_cls is not None:
            assert np.array_equal(out.e_cls[i].cpu().numpy().astype(np.int64), r["e_cls"]), tag + " E_P"
        if out.best_chain is not None:
            assert out.best_chain[i].item() == r["best_chain"], tag + " best chain"
        assert np.array_equal(rec[i], r["recovery"]), tag + " recovery"
        if out.paper_recovery is not None:
            assert np.array_equal(out.paper_recovery[i].cpu().numpy(), r["paper_recovery"]), tag + " R0 L_P*"
