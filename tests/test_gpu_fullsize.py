"""Parity at the measured workload shapes, in the launch configuration the
benchmark times (all groups of a workload in one persistent launch, captured
in a hipGraph where the benchmark uses one).  The oracle recomputes sampled
syndromes end to end, or sampled chains where a whole syndrome would take it
minutes; every syndrome of the launch is also checked for properties that hold
at any size (syndrome-consistent recovery of energy E_best in coset P*)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_17837_amd import _lib as X
from paper_2509_17837_amd import decoder as D
from paper_2509_17837_amd import inputs
from tests._parity import pool

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


def oracle_syndromes(wl, seeds, outs, meta, picks):
    """Full oracle decode of the picked (group, syndrome) pairs."""
    sched = wl["schedule"]
    beta = O.schedule(inputs.SCHEDULE_KIND[sched[0]], sched[1], sched[2], wl["sweeps"])

    def one(job):
        gi, i = job
        m = meta[gi]
        lat = O.Lattice(m["layout"], m["d"])
        w, wg = O.weights(m["p"], O.noise(m["p"], m["eta"], m["conv"]))
        return lat.decode(w, wg, m["syn"][i], int(m["uid"][i]), wl["n_rep"], beta, seeds["greedy"],
                          seeds["anneal"], chains=True)

    for (gi, i), r in zip(picks, pool().map(one, picks)):
        o = outs[gi]
        tag = f"group {gi} syndrome {i}"
        assert np.array_equal(o.refs[i].cpu().numpy(), r["refs"]), tag
        assert np.array_equal(o.chain_emin[i].cpu().numpy(), r["chain_emin"]), tag
        assert np.array_equal(o.chain_stop[i].cpu().numpy(), r["chain_stop"]), tag
        assert np.array_equal(o.chain_e[i].cpu().numpy(), r["chain_e"]), tag
        assert o.e_best[i].item() == r["e_best"] and o.cls[i].item() == r["cls"], tag
        assert np.array_equal(o.recovery[i].cpu().numpy(), r["recovery"]), tag


def oracle_chains(wl, seeds, outs, meta, picks):
    """Oracle greedy reference and single-chain annealing of picked chains."""
    sched = wl["schedule"]
    beta = O.schedule(inputs.SCHEDULE_KIND[sched[0]], sched[1], sched[2], wl["sweeps"])

    def one(job):
        gi, i, c = job
        m = meta[gi]
        lat = O.Lattice(m["layout"], m["d"])
        w, wg = O.weights(m["p"], O.noise(m["p"], m["eta"], m["conv"]))
        ref = lat.greedy(wg, m["syn"][i], int(m["uid"][i]), c // 4, seeds["greedy"])
        res = lat.anneal_chain(w, beta, seeds["anneal"], int(m["uid"][i]), c, ref ^ lat.logical(c % 4),
                               want_snap=False)
        return ref, res

    for (gi, i, c), (ref, r) in zip(picks, pool().map(one, picks)):
        o = outs[gi]
        tag = f"group {gi} syndrome {i} chain {c}"
        assert np.array_equal(o.refs[i, c // 4].cpu().numpy(), ref), tag
        assert o.chain_emin[i, c].item() == r["emin"], tag
        assert o.chain_stop[i, c].item() == r["stop"], tag
        assert o.chain_e[i, c].item() == r["e"], tag


def test_d11_full_launch():
    wl, seeds, outs, meta = build_launch("d11_bias100", 2048, graph=True)
    check_properties(wl, outs, meta)
    picks = [(g, i) for g in range(len(outs)) for i in (0, 777, 2047)]
    oracle_syndromes(wl, seeds, outs, meta, picks)


def test_mixed_distances_full_launch():
    wl, seeds, outs, meta = build_launch("mixed_d5_21", 96, graph=True)
    check_properties(wl, outs, meta)
    rng = np.random.default_rng(5)
    picks = [(g, int(rng.integers(96)), int(rng.integers(4 * wl["n_rep"]))) for g in range(len(outs)) for _ in range(4)]
    oracle_chains(wl, seeds, outs, meta, picks)
    oracle_syndromes(wl, seeds, outs, meta, [(0, 3), (1, 50)])


def test_d31_full_launch():
    wl, seeds, outs, meta = build_launch("d31_large", 2, graph=False)
    check_properties(wl, outs, meta)
    rng = np.random.default_rng(6)
    picks = [(int(rng.integers(1)), int(rng.integers(2)), int(rng.integers(4 * wl["n_rep"]))) for _ in range(12)]
    oracle_chains(wl, seeds, outs, meta, picks)


def test_planar_paper_full_launch():
    """The paper's own set-up: planar layout, 1:eta:1 channel, log schedule
    0.9 beta_N -> beta_N over N_beta = 100, N_SA = 10; six (p, eta) groups of
    2048 syndromes in one captured launch, as the benchmark times them."""
    wl, seeds, outs, meta = build_launch("planar_paper_d9", 2048, graph=True)
    check_properties(wl, outs, meta)
    picks = [(g, i) for g in range(len(outs)) for i in (0, 1, 1023, 2047)]
    oracle_syndromes(wl, seeds, outs, meta, picks)
