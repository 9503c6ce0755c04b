"""Parity at the measured workload shapes, in the launch configuration the
benchmark times (all groups of a workload in one persistent launch, captured
in a hipGraph).  The oracle decodes the leading syndromes of every group end
to end -- 200 per p at d = 11, 20 per distance in the mixed launch, 4 at
d = 31 -- and every chain of those syndromes is compared (E_min, the phase of
the minimum, final energy), with the references, their classes, E_P, P*, the
best chain and the recovery.  Every syndrome of the launch is also checked
for properties that hold at any size (syndrome-consistent recovery of energy
E_best in coset P*)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_17837_amd import _lib as X
from paper_2509_17837_amd import decoder as D
from paper_2509_17837_amd import inputs
from tests._parity import oracle_decode_by_chain, pool

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    X.lib()


def build_launch(name, n_per_group, graph):
    wl = inputs.WORKLOADS[name]
    seeds = inputs.seeds(name)
    kind = inputs.SCHEDULE_KIND[wl["schedule"][0]]
    beta = D.schedule(kind, wl["schedule"][1], wl["schedule"][2], wl["sweeps"])
    specs = [(d, p, eta) for d in wl["d"] for p in wl["p"] for eta in wl["eta"]]
    layout, conv = inputs.layout_of(wl), inputs.convention_of(wl)
    groups, outs, meta = [], [], []
    for gi, (d, p, eta) in enumerate(specs):
        lat = D.Lattice(layout, d)
        w, wg = D.weights(p, D.noise(p, eta, conv))
        plan = D.Plan(lat, w, wg, beta)
        olat = O.Lattice(layout, d)
        err = inputs.sample_errors(n_per_group, lat.nq, inputs.channel(p, eta, conv), seeds["sample"], stream=gi)
        syn = np.stack([olat.syndrome(e) for e in err])
        uid = inputs.sample_uids(n_per_group, gi * n_per_group)
        g, o = D.make_group(plan, wl["n_rep"], torch.from_numpy(uid.view(np.int32)).cuda(),
                            syn=torch.from_numpy(syn).cuda(), want_chains=True)
        groups.append(g)
        outs.append(o)
        meta.append(dict(d=d, p=p, eta=eta, layout=layout, conv=conv, syn=syn, uid=uid, olat=olat, lat=lat, plan=plan))
    print(f"[fullsize] {name}: {len(groups)} groups x {n_per_group} syndromes, R={wl['n_rep']}, "
          f"sweeps={wl['sweeps']}, graph={graph}", flush=True)
    if graph:
        G = D.Graph(groups, seeds["greedy"], seeds["anneal"])
        G.launch()
        G.stream.synchronize()
    else:
        D.decode_groups(groups, seeds["greedy"], seeds["anneal"])
        torch.cuda.synchronize()
    return wl, seeds, outs, meta


def check_properties(wl, outs, meta):
    for o, m in zip(outs, meta):
        rec = o.recovery.cpu().numpy()
        eb = o.e_best.cpu().numpy()
        cls = o.cls.cpu().numpy()
        refs0 = o.refs[:, 0].cpu().numpy()
        w = O.weights(m["p"], O.noise(m["p"], m["eta"], m["conv"]))[0]
        emin = o.chain_emin.cpu().numpy()
        for i in range(len(rec)):
            assert np.array_equal(m["olat"].syndrome(rec[i]), m["syn"][i])
            assert m["olat"].energy(w, rec[i]) == eb[i]
            assert m["olat"].cls(rec[i], refs0[i]) == cls[i]
            assert eb[i] == emin[i].min()


def compare_syndrome(o, i, r, tag):
    assert np.array_equal(o.refs[i].cpu().numpy(), r["refs"]), tag + " refs"
    assert np.array_equal(o.qcls[i].cpu().numpy(), r["qcls"]), tag + " classes"
    assert np.array_equal(o.chain_emin[i].cpu().numpy(), r["chain_emin"]), tag + " chain E_min"
    assert np.array_equal(o.chain_stop[i].cpu().numpy(), r["chain_stop"]), tag + " chain stop"
    assert np.array_equal(o.chain_e[i].cpu().numpy(), r["chain_e"]), tag + " chain E"
    assert np.array_equal(o.e_cls[i].cpu().numpy().astype(np.int64), r["e_cls"]), tag + " E_P"
    assert o.e_best[i].item() == r["e_best"] and o.cls[i].item() == r["cls"], tag + " E_best, P*"
    assert o.best_chain[i].item() == r["best_chain"], tag + " best chain"
    assert np.array_equal(o.recovery[i].cpu().numpy(), r["recovery"]), tag + " recovery"
    if "paper_recovery" in r:
        assert np.array_equal(o.paper_recovery[i].cpu().numpy(), r["paper_recovery"]), tag + " R_0 L_P*"


def oracle_syndromes(wl, seeds, outs, meta, picks):
    """Full oracle decode of the picked (group, syndrome) pairs, one syndrome
    per host thread, the largest lattices first."""
    sched = wl["schedule"]
    beta = O.schedule(inputs.SCHEDULE_KIND[sched[0]], sched[1], sched[2], wl["sweeps"])
    picks = sorted(picks, key=lambda j: -meta[j[0]]["olat"].nstab)

    def one(job):
        gi, i = job
        m = meta[gi]
        lat = O.Lattice(m["layout"], m["d"])
        w, wg = O.weights(m["p"], O.noise(m["p"], m["eta"], m["conv"]))
        return lat.decode(w, wg, m["syn"][i], int(m["uid"][i]), wl["n_rep"], beta, seeds["greedy"],
                          seeds["anneal"], chains=True)

    print(f"[fullsize] oracle on {len(picks)} syndromes", flush=True)
    for (gi, i), r in zip(picks, pool().map(one, picks)):
        compare_syndrome(outs[gi], i, r, f"group {gi} syndrome {i}")


def test_d11_full_launch():
    """The headline launch: four p groups of 2048 syndromes (d = 11, 32
    replicas, 2000 sweeps) captured in one graph; the oracle decodes the
    first 200 syndromes of every p (800 syndromes, 102400 chains).  Against
    the mathematics directly (Eqs. (18)-(21)): on those syndromes every E_P
    bounds the exact minimum of its coset (frontier program,
    tests/_exact_dp.c) from above, and the syndromes decoded to the exact
    least minimum clear the binomial bar of the rate calibrated at this
    distance (tests/golden/hit_rate_calibration_d11.py)."""
    import os

    from tests import _exact, _hitrate
    wl, seeds, outs, meta = build_launch("d11_bias100", 2048, graph=True)
    check_properties(wl, outs, meta)
    n = 200
    oracle_syndromes(wl, seeds, outs, meta, [(g, i) for g in range(len(outs)) for i in range(n)])
    cal = _hitrate.read_calibration(os.path.join(os.path.dirname(__file__), "golden", "hit_rates_d11.txt"))
    for gi, (o, m) in enumerate(zip(outs, meta)):
        refs0 = o.refs[:n, 0].cpu().numpy()
        e_cls = o.e_cls[:n].cpu().numpy().astype(np.int64)
        e_best = o.e_best[:n].cpu().numpy()
        w = O.weights(m["p"], O.noise(m["p"], m["eta"], m["conv"]))[0]
        lat = m["olat"]

        def exact(i):
            return [_exact.coset_minimum_c(lat.fq, lat.fm, refs0[i] ^ lat.logical(P), w) for P in range(4)]

        ex = np.array(list(pool().map(exact, range(n))), np.int64)
        assert (e_cls >= ex).all(), f"p={m['p']}: E_P below an exact coset minimum"
        hits = int((e_best == ex.min(axis=1)).sum())
        print(f"[fullsize] d11 p={m['p']}: {hits}/{n} syndromes at the exact least coset minimum", flush=True)
        assert hits >= _hitrate.bar(*cal[f"rotated_d11_p{m['p']:.2f}"], n)


def test_mixed_distances_full_launch():
    """One launch of d = 5, 9, 13, 17, 21 (256 syndromes each, 64 replicas,
    5000 sweeps); the oracle decodes the first 20 syndromes of every
    distance."""
    wl, seeds, outs, meta = build_launch("mixed_d5_21", 256, graph=True)
    check_properties(wl, outs, meta)
    oracle_syndromes(wl, seeds, outs, meta, [(g, i) for g in range(len(outs)) for i in range(20)])


def test_d31_full_launch():
    """d = 31, 128 replicas (512 chains), 10^4 sweeps of the geometric
    schedule 0.02 -> 20 (checkpoints every 313 sweeps), 16 syndromes in one
    captured launch; the oracle decodes the first 4 syndromes, each one's 512
    chains spread over the host threads."""
    wl, seeds, outs, meta = build_launch("d31_large", 16, graph=True)
    check_properties(wl, outs, meta)
    m = meta[0]
    sched = wl["schedule"]
    beta = O.schedule(inputs.SCHEDULE_KIND[sched[0]], sched[1], sched[2], wl["sweeps"])
    w, wg = O.weights(m["p"], O.noise(m["p"], m["eta"], m["conv"]))
    for i in range(4):
        print(f"[fullsize] d31 oracle syndrome {i}", flush=True)
        r = oracle_decode_by_chain(m["layout"], m["d"], w, wg, m["syn"][i], m["uid"][i], wl["n_rep"], beta,
                                   seeds["greedy"], seeds["anneal"])
        compare_syndrome(outs[0], i, r, f"d31 syndrome {i}")


def test_planar_paper_full_launch():
    """The paper's own set-up: planar layout, 1:eta:1 channel, log schedule
    0.9 beta_N -> beta_N over N_beta = 100, N_SA = 10; six (p, eta) groups of
    2048 syndromes in one captured launch, as the benchmark times them."""
    wl, seeds, outs, meta = build_launch("planar_paper_d9", 2048, graph=True)
    check_properties(wl, outs, meta)
    picks = [(g, i) for g in range(len(outs)) for i in (0, 1, 1023, 2047)]
    oracle_syndromes(wl, seeds, outs, meta, picks)
