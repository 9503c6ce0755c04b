"""Serving loop (continuous batching): a request decoded alone, in a mix of
other requests of different distance and bias that arrive while it is on the
device, and by the batch decoder all give identical results (bit for bit),
which also match the oracle; admission respects the slot and queue limits."""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_17837_amd import _lib as X
from paper_2509_17837_amd import decoder as D
from paper_2509_17837_amd import inputs

pytestmark = pytest.mark.gpu

GS, AS = 0xC0FFEE, 0xBADC0DE


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    X.lib()


class Spec:
    def __init__(self, d, p, eta, sweeps, n, stream, uid0, layout=X.ROTATED, conv=0,
                 sched=(X.SCHED_GEOMETRIC, 0.05, 10.0)):
        self.d, self.p, self.eta, self.sweeps, self.conv, self.sched = d, p, eta, sweeps, conv, sched
        self.lat = D.Lattice(layout, d)
        w, wg = D.weights(p, D.noise(p, eta, conv))
        beta = D.schedule(sched[0], sched[1], sched[2], sweeps)
        self.plan = D.Plan(self.lat, w, wg, beta)
        self.olat = O.Lattice(layout, d)
        err = inputs.sample_errors(n, self.lat.nq, inputs.channel(p, eta, conv), 77, stream=stream)
        self.syn = np.stack([self.olat.syndrome(e) for e in err])
        self.uid = inputs.sample_uids(n, uid0)

    def batch(self, n_rep):
        out = D.decode(self.plan, torch.from_numpy(self.syn).cuda(), torch.from_numpy(self.uid.view(np.int32)).cuda(),
                       n_rep, GS, AS)
        torch.cuda.synchronize()
        return out


def same(res, out, i):
    return (res["e_best"] == out.e_best[i].item() and res["cls"] == out.cls[i].item() and
            np.array_equal(res["recovery"], out.recovery[i].cpu().numpy()) and
            res["e_cls"] == out.e_cls[i].cpu().tolist())


@pytest.mark.parametrize("lanes,waves", [(0, 0), (1, 0), (64, 0), (16, 30)],
                         ids=["adaptive", "plan-kernel", "up-to-64-lanes", "lanes-shift-with-load"])
def test_request_alone_and_in_mix(lanes, waves):
    """lanes/waves: the per-slice lanes-per-chain policy; with a small wave
    budget the lane count of a resident request changes as others arrive and
    leave, which must not change its result."""
    R = 16
    specs = [Spec(d, 0.12, eta, 300, 6, k, 1000 * k)
             for k, (d, eta) in enumerate([(7, 1.0), (11, 10.0), (15, 1000.0), (19, 10.0), (25, 1.0), (11, 1000.0)])]
    target = specs[1]
    srv = D.Server(max_slots=32, max_rep=R, max_qubits=625, sweeps_per_slice=40, greedy_seed=GS, anneal_seed=AS,
                   max_lanes_per_chain=lanes, max_waves=waves)
    # alone
    t = srv.submit(target.plan, target.syn[0], target.uid[0], R)
    srv.drain()
    alone = srv.poll(t)
    assert alone is not None
    # in a mix: requests keep arriving while earlier ones are resident
    tickets = []
    rng = np.random.default_rng(1)
    order = [(k, i) for k in range(len(specs)) for i in range(len(specs[k].uid))]
    rng.shuffle(order)
    for n, (k, i) in enumerate(order):
        tickets.append((k, i, srv.submit(specs[k].plan, specs[k].syn[i], specs[k].uid[i], R)))
        if n % 7 == 3:
            time.sleep(0.002)
    srv.drain()
    results = {(k, i): srv.poll(tk) for k, i, tk in tickets}
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(order) + 1 and st["slices"] > 1
    mixed = results[(1, 0)]
    for key in ("e_best", "cls", "e_cls"):
        assert alone[key] == mixed[key]
    assert np.array_equal(alone["recovery"], mixed["recovery"])
    # every served result equals the batch decoder's
    for k, s in enumerate(specs):
        out = s.batch(R)
        for i in range(len(s.uid)):
            assert same(results[(k, i)], out, i), f"spec {k} request {i}"
    # and the oracle's, on a sample
    for k, i in [(0, 2), (1, 0), (4, 5)]:
        s = specs[k]
        w, wg = O.weights(s.p, O.noise(s.p, s.eta))
        beta = O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, s.sweeps)
        ref = s.olat.decode(w, wg, s.syn[i], int(s.uid[i]), R, beta, GS, AS)
        r = results[(k, i)]
        assert r["e_best"] == ref["e_best"] and r["cls"] == ref["cls"]
        assert np.array_equal(r["recovery"], ref["recovery"])


def test_admission_limits():
    """Two slots and a tiny queue: submissions beyond the queue are refused
    with EAGAIN, admitted work completes, and results still match."""
    R = 4
    s = Spec(9, 0.15, 10.0, 120, 12, 9, 500)
    srv = D.Server(max_slots=2, max_rep=R, max_qubits=81, sweeps_per_slice=30, max_pending=3, greedy_seed=GS,
                   anneal_seed=AS)
    got, refused = {}, 0
    for i in range(len(s.uid)):
        while True:
            t = srv.try_submit(s.plan, s.syn[i], s.uid[i], R)
            if t is not None:
                got[i] = t
                break
            refused += 1
            time.sleep(0.001)
    srv.drain()
    res = {i: srv.poll(t) for i, t in got.items()}
    st = srv.stats()
    srv.close()
    assert refused > 0 and st["rejected"] == refused
    out = s.batch(R)
    for i in range(len(s.uid)):
        assert same(res[i], out, i)
    assert st["p99_latency_s"] >= st["p50_latency_s"] > 0


def test_submit_many():
    """Requests queued in one call (xzzx_server_submit_many) are served like
    single submissions; a request that does not fit stops the batch there
    (EINVAL, the requests before it queued), and a full queue stops it with
    EAGAIN."""
    R = 4
    a = Spec(7, 0.15, 10.0, 60, 6, 21, 900)
    b = Spec(11, 0.2, 100.0, 60, 5, 22, 950)
    srv = D.Server(max_slots=4, max_rep=R, max_qubits=121, sweeps_per_slice=20, greedy_seed=GS, anneal_seed=AS)
    plans = [a.plan] * len(a.uid) + [b.plan] * len(b.uid)
    syns = list(a.syn) + list(b.syn)
    uids = list(a.uid) + list(b.uid)
    tickets = srv.submit_many(plans, syns, uids, R)
    assert len(set(tickets)) == len(plans)
    srv.drain()
    res = [srv.poll(t) for t in tickets]
    oa, ob = a.batch(R), b.batch(R)
    for i in range(len(a.uid)):
        assert same(res[i], oa, i)
    for i in range(len(b.uid)):
        assert same(res[len(a.uid) + i], ob, i)
    # a 13 x 13 lattice does not fit max_qubits = 121: the batch stops there
    big = Spec(13, 0.15, 10.0, 10, 1, 23, 990)
    with pytest.raises(X.XzzxError) as e:
        srv.submit_many([a.plan, big.plan, a.plan], [a.syn[0], big.syn[0], a.syn[1]], [1, 2, 3], R)
    assert e.value.rc == X.XZZX_EINVAL
    srv.drain()
    assert srv.stats()["submitted"] == len(plans) + 1
    srv.close()
    small = D.Server(max_slots=1, max_rep=R, max_qubits=49, sweeps_per_slice=20, max_pending=2,
                     greedy_seed=GS, anneal_seed=AS)
    with pytest.raises(X.XzzxError) as e:
        small.submit_many([a.plan] * 6, list(a.syn), list(a.uid), R)
    assert e.value.rc == X.XZZX_EAGAIN
    small.drain()
    small.close()


def test_byte_kernel_and_empty_schedule():
    """Requests on the byte-state kernel (planar-free path via set_kernel) and
    with an empty schedule are served like the batch decoder serves them."""
    R = 2
    a = Spec(7, 0.2, 10.0, 50, 3, 21, 40)
    a.plan.set_kernel(X.KERNEL_BYTES)
    b = Spec(5, 0.2, 10.0, 0, 3, 22, 80)
    srv = D.Server(max_slots=8, max_rep=R, max_qubits=49, sweeps_per_slice=17, greedy_seed=GS, anneal_seed=AS)
    tk = [(a, i, srv.submit(a.plan, a.syn[i], a.uid[i], R)) for i in range(3)]
    tk += [(b, i, srv.submit(b.plan, b.syn[i], b.uid[i], R)) for i in range(3)]
    srv.drain()
    res = [(s, i, srv.poll(t)) for s, i, t in tk]
    srv.close()
    outs = {id(a): a.batch(R), id(b): b.batch(R)}
    for s, i, r in res:
        assert same(r, outs[id(s)], i)
    with pytest.raises(X.XzzxError):
        D.Server(max_slots=0)
    with pytest.raises(X.XzzxError):
        D.Server(max_lanes_per_chain=3)
    with pytest.raises(X.XzzxError):
        D.Server(max_lanes_per_chain=128)


@pytest.mark.parametrize("slice_sweeps", [1000, 100])
def test_replay_from_states_kept_while_serving(slice_sweeps):
    """The byte-state serving kernel keeps each chain's state every 64 sweeps
    inside a slice (1000: the whole 300-sweep schedule in one slice; 100:
    slice starts and one kept state per slice), and the best chain's replay
    starts from the last kept state before its E_min phase; recoveries equal
    the batch decoder's and the oracle's."""
    R = 16
    s = Spec(11, 0.12, 10.0, 300, 4, 31, 9000)
    srv = D.Server(max_slots=8, max_rep=R, max_qubits=121, sweeps_per_slice=slice_sweeps, greedy_seed=GS,
                   anneal_seed=AS, max_lanes_per_chain=64)
    tk = [srv.submit(s.plan, s.syn[i], s.uid[i], R) for i in range(4)]
    srv.drain()
    res = [srv.poll(t) for t in tk]
    srv.close()
    out = s.batch(R)
    for i, r in enumerate(res):
        assert same(r, out, i), f"request {i}"
    w, wg = O.weights(s.p, O.noise(s.p, s.eta))
    beta = O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, s.sweeps)
    ref = s.olat.decode(w, wg, s.syn[0], int(s.uid[0]), R, beta, GS, AS)
    assert res[0]["e_best"] == ref["e_best"] and np.array_equal(res[0]["recovery"], ref["recovery"])


def test_every_specialised_serving_class():
    """With one lane per chain every request runs on the specialised
    packed-row serving kernels, one launch per register class; distances
    from every class (d = 3..15 but 9, 9, 17-21, 23-25, 27-29, 31) are served
    together and each result equals the batch decoder's."""
    R = 16
    specs = [Spec(d, 0.12, 10.0, 40, 2, 40 + d, 20000 + 100 * d) for d in (5, 9, 13, 17, 21, 23, 27, 29, 31)]
    srv = D.Server(max_slots=32, max_rep=R, max_qubits=961, sweeps_per_slice=15, greedy_seed=GS, anneal_seed=AS,
                   max_lanes_per_chain=1)
    tk = [(s, i, srv.submit(s.plan, s.syn[i], s.uid[i], R)) for s in specs for i in range(2)]
    srv.drain()
    res = [(s, i, srv.poll(t)) for s, i, t in tk]
    st = srv.stats()
    srv.close()
    assert st["slices"] > 1
    outs = {id(s): s.batch(R) for s in specs}
    for s, i, r in res:
        assert same(r, outs[id(s)], i), f"d={s.d} request {i}"


@pytest.mark.parametrize("lanes", [0, 1, 64], ids=["adaptive", "plan-kernel", "up-to-64-lanes"])
def test_planar_requests(lanes):
    """The paper's set-up served: planar d = 5, 7, 9, p_x:p_y:p_z = 1:eta:1, log
    schedule over N_beta = 100, N_SA = 10.  The server runs them on the
    generic packed-row or the byte-state serving kernels; every result equals
    the batch decoder's (the planar kernel specialised to d) and, on a
    sample, the oracle's."""
    R = 10
    specs = [Spec(d, 0.15, eta, 100, 3, 60 + d, 30000 + 100 * d, layout=X.PLANAR, conv=1,
                  sched=(X.SCHED_PAPER_LOG, 0.9, 1.0)) for d, eta in ((5, 1.0), (7, 5.0), (9, 10.0))]
    srv = D.Server(max_slots=16, max_rep=R, max_qubits=145, sweeps_per_slice=30, greedy_seed=GS, anneal_seed=AS,
                   max_lanes_per_chain=lanes)
    tk = [(s, i, srv.submit(s.plan, s.syn[i], s.uid[i], R)) for s in specs for i in range(3)]
    srv.drain()
    res = [(s, i, srv.poll(t)) for s, i, t in tk]
    srv.close()
    outs = {id(s): s.batch(R) for s in specs}
    for s, i, r in res:
        assert same(r, outs[id(s)], i), f"planar d={s.d} request {i}"
    s = specs[2]
    w, wg = O.weights(s.p, O.noise(s.p, s.eta, 1))
    beta = O.schedule(O.SCHED_PAPER_LOG, 0.9, 1.0, s.sweeps)
    ref = s.olat.decode(w, wg, s.syn[1], int(s.uid[1]), R, beta, GS, AS)
    r = [x for t, i, x in res if t is s and i == 1][0]
    assert r["e_best"] == ref["e_best"] and np.array_equal(r["recovery"], ref["recovery"])


def test_serving_workload_requests_match_oracle():
    """The serving workload at its real sizes: 200 single-syndrome requests
    (d in {7, 11, 15, 19, 25} and eta in {1, 10, 1000} drawn per request,
    p = 0.12, 16 replicas, 1000 sweeps of the geometric schedule 0.05 -> 10)
    arriving as a Poisson stream at 10^4 per second, so that many are resident
    at once and join while others run; every served result (E_best, P*, E_P,
    recovery) equals the oracle's decode of that request."""
    from paper_2509_17837_amd import inputs as I
    from tests._parity import pool
    name = "serving_d7_25"
    wl = I.WORKLOADS[name]
    seeds = I.seeds(name)
    R, sweeps, p = wl["n_rep"], wl["sweeps"], wl["p"][0]
    specs = [(d, eta) for d in wl["d"] for eta in wl["eta"]]
    plans = {k: Spec(d, p, eta, sweeps, 1, 900 + k, 0).plan for k, (d, eta) in enumerate(specs)}
    olats = {d: O.Lattice(O.ROTATED, d) for d in wl["d"]}
    n = 200
    rng = np.random.default_rng([seeds["sample"], 12])
    pick = rng.integers(0, len(specs), size=n)
    reqs = []
    for i in range(n):
        d, eta = specs[pick[i]]
        err = I.sample_errors(1, d * d, I.channel(p, eta), seeds["sample"], stream=200000 + i)[0]
        reqs.append((int(pick[i]), olats[d].syndrome(err), 8_000_000 + i))
    arrivals = I.poisson_arrivals(1e4, n, seeds["sample"] + 5)
    srv = D.Server(max_slots=256, max_rep=R, max_qubits=625, sweeps_per_slice=400, greedy_seed=seeds["greedy"],
                   anneal_seed=seeds["anneal"])
    print(f"[serving] {n} requests of {name} at 1e4/s", flush=True)
    t0 = time.perf_counter()
    tickets = []
    for i, (k, syn, uid) in enumerate(reqs):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        tickets.append(srv.submit(plans[k], syn, uid, R))
    srv.drain()
    got = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == n and st["slices"] > 1
    beta = O.schedule(O.SCHED_GEOMETRIC, 0.05, 10.0, sweeps)

    def oracle(job):
        k, syn, uid = job
        d, eta = specs[k]
        w, wg = O.weights(p, O.noise(p, eta))
        return O.Lattice(O.ROTATED, d).decode(w, wg, syn, uid, R, beta, seeds["greedy"], seeds["anneal"])

    order = sorted(range(n), key=lambda i: -specs[reqs[i][0]][0])
    refs = dict(zip(order, pool().map(oracle, [reqs[i] for i in order])))
    for i in range(n):
        r, g = refs[i], got[i]
        tag = f"request {i} (d={specs[reqs[i][0]][0]}, eta={specs[reqs[i][0]][1]})"
        assert g["e_best"] == r["e_best"] and g["cls"] == r["cls"], tag
        assert g["e_cls"] == list(r["e_cls"]), tag
        assert np.array_equal(g["recovery"], r["recovery"]), tag
