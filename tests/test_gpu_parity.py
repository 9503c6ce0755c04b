"""Bit-exact parity of the HIP path (through the C ABI) with the oracle.

Every integer output is compared element by element: greedy references and
their classes, per-chain E_min / phase of the minimum / final energy / final
state, per-coset minima, P*, the best chain, the minimum-energy recovery and
R_0 L_P*.  Sizes span several wavefront tasks with ragged tails; the full
workload shapes are covered by sampled chains (test_gpu_fullsize.py)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_17837_amd import _lib as X
from paper_2509_17837_amd import decoder as D
from paper_2509_17837_amd import inputs
from tests._parity import Problem, compare_decode, gpu_plan, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    X.lib()
    torch.cuda.synchronize()


def run_decode(prob, plan=None, flags=0, mode=X.GREEDY_RANDOM, want_final=True):
    plan = plan or gpu_plan(prob)
    print(f"[decode] layout={prob.layout} d={prob.d} n_syn={prob.n_syn} R={prob.n_rep} "
          f"sweeps={prob.n_sweeps} lanes={plan.info()['lanes_per_chain']} flags={flags}", flush=True)
    out = D.decode(plan, to_dev(prob.syn), to_dev(prob.uid.view(np.int32)), prob.n_rep, prob.greedy_seed,
                   prob.anneal_seed, greedy_mode=mode, flags=flags, want_chains=True, want_final=want_final)
    torch.cuda.synchronize()
    return out


def test_syndrome_kernel():
    for layout, d in [(0, 3), (0, 11), (0, 31), (1, 5), (1, 9)]:
        prob = Problem(layout, d, 0.2, 3.0, 97, 1, 0)
        plan = gpu_plan(prob)
        rng = np.random.default_rng(d)
        cfg = rng.integers(0, 4, (97, prob.olat.nq)).astype(np.uint8)
        got = D.syndrome(plan, to_dev(cfg)).cpu().numpy()
        assert np.array_equal(got, prob.olat.syndrome(cfg))


@pytest.mark.parametrize("layout,d,p,eta", [(0, 3, 0.15, 10.0), (0, 11, 0.25, 100.0), (0, 15, 0.3, 1.0),
                                            (0, 17, 0.2, 10.0), (0, 21, 0.18, 10.0), (0, 31, 0.2, 10.0),
                                            (1, 7, 0.1, 1.0)])
@pytest.mark.parametrize("mode", [X.GREEDY_RANDOM, X.GREEDY_SAME, X.GREEDY_BOUNDARY])
def test_greedy_kernel(layout, d, p, eta, mode):
    """References of the GPU greedy kernel equal the oracle's byte for byte.
    Up to 128 nodes per colour (rotated d <= 15) each half wavefront matches
    one colour (d = 15 at p = 0.3: several defects per lane); beyond, the
    colours take the whole wavefront in turn."""
    n_syn, R = (12, 5) if d < 31 else (3, 4)
    prob = Problem(layout, d, p, eta, n_syn, R, 0, seed=d + 3)
    plan = gpu_plan(prob)
    refs, qcls = D.greedy_init(plan, to_dev(prob.syn), to_dev(prob.uid.view(np.int32)), R, prob.greedy_seed, mode)
    refs = refs.cpu().numpy()
    qcls = qcls.cpu().numpy()
    for i in range(n_syn):
        for r in range(R):
            exp = prob.oracle_greedy(i, r, mode)
            assert np.array_equal(refs[i, r], exp), f"syndrome {i} replica {r}"
            assert qcls[i, r] == prob.olat.cls(refs[i, r], refs[i, 0])


def test_greedy_beyond_one_launch():
    """More (syndrome, replica) pairs than one launch can address (2^32
    work-items = 67108863 wavefronts): the greedy references go in chunks;
    pairs sampled on both sides of the chunk boundary equal the oracle's."""
    n_syn, R = 1_000_000, 70
    prob = Problem(0, 3, 0.15, 10.0, 0, R, 0, seed=4)
    plan = gpu_plan(prob)
    err = inputs.sample_errors(n_syn, prob.olat.nq, inputs.channel(0.15, 10.0), 91, stream=3)
    syn = D.syndrome(plan, to_dev(err))
    uid = to_dev(inputs.sample_uids(n_syn).view(np.int32))
    print(f"[greedy] {n_syn} syndromes x {R} replicas", flush=True)
    refs, _ = D.greedy_init(plan, syn, uid, R, prob.greedy_seed, X.GREEDY_RANDOM)
    torch.cuda.synchronize()
    syn_h = syn.cpu().numpy()
    boundary = (2**32 - 1) // 64
    picks = [(0, 0), (boundary // R - 1, R - 1), (boundary // R, boundary % R), (boundary // R, R - 1),
             (n_syn - 1, 0), (n_syn - 1, R - 1), (777_777, 33)]
    for s, r in picks:
        exp = prob.olat.greedy(prob.wg, syn_h[s], s, r, prob.greedy_seed, O.GREEDY_RANDOM)
        got = refs[s, r].cpu().numpy()
        assert np.array_equal(got, exp), (s, r)
        assert np.array_equal(prob.olat.syndrome(got), syn_h[s])


@pytest.mark.parametrize("layout,d", [(0, 7), (1, 5)])
def test_decode_against_exact_minima(layout, d):
    """The GPU decoder (default kernels: specialised packed rows) against the
    mathematics directly: every coset estimate E_P bounds the exact coset
    minimum (a frontier dynamic program over the generator bits) from above,
    and a slow schedule reaches the exact least minimum."""
    from tests import _exact
    prob = Problem(layout, d, 0.12, 10.0, 6, 16, 400, sched=("linear", 0.1, 5.0), seed=70 + d)
    out = run_decode(prob)
    e_cls = out.e_cls.cpu().numpy()
    refs0 = out.refs[:, 0].cpu().numpy()
    hits = 0
    for i in range(prob.n_syn):
        exact = [_exact.coset_minimum(prob.olat.fq, prob.olat.fm, refs0[i] ^ prob.olat.logical(P), prob.w)
                 for P in range(4)]
        assert all(int(e_cls[i, P]) >= exact[P] for P in range(4)), i
        hits += int(out.e_best[i].item()) == min(exact)
    assert hits >= prob.n_syn - 1


def test_decode_small_d3_all():
    """Distance 3, one replica, 200 linear sweeps, 1000 syndromes."""
    prob = Problem(0, 3, 0.15, 10.0, 1000, 1, 200, sched=("linear", 0.1, 5.0), seed=1000)
    out = run_decode(prob)
    compare_decode(prob, out, prob.oracle_decode())


@pytest.mark.parametrize("p", [0.10, 0.25])
def test_decode_d11(p):
    prob = Problem(0, 11, p, 100.0, 24, 32, 150, seed=int(p * 100))
    out = run_decode(prob)
    compare_decode(prob, out, prob.oracle_decode())


@pytest.mark.parametrize("layout,d", [(1, 5), (1, 7), (0, 5), (0, 9)])
def test_decode_layouts(layout, d):
    prob = Problem(layout, d, 0.12, 5.0, 40, 3, 60, seed=d)
    out = run_decode(prob)
    compare_decode(prob, out, prob.oracle_decode())


@pytest.mark.parametrize("d,eta,n_beta", [(5, 1.0, 100), (9, 5.0, 100), (9, 10.0, 100), (9, 10.0, 7), (7, 5.0, 1)])
@pytest.mark.parametrize("mode", [X.GREEDY_RANDOM, X.GREEDY_SAME, X.GREEDY_BOUNDARY])
def test_paper_setup(d, eta, n_beta, mode):
    """The paper's own set-up (Sec. V): planar layout, p_x:p_y:p_z = 1:eta:1,
    log schedule 0.9 beta_N -> beta_N over N_beta sweeps (Eqs. 23-24, gamma = 0
    at N_beta = 1), N_SA = 10, each reference construction of Sec. V.C."""
    prob = Problem(1, d, 0.15, eta, 24, 10, n_beta, sched=("paper_log", 0.9, 1.0), seed=40 + d + n_beta, conv=1)
    out = run_decode(prob, mode=mode)
    compare_decode(prob, out, prob.oracle_decode(mode=mode))


@pytest.mark.parametrize("layout,d,n_syn,R,sweeps", [(0, 3, 200, 1, 50), (0, 11, 21, 7, 30), (0, 31, 2, 16, 4),
                                                     (1, 9, 30, 10, 100), (1, 5, 70, 3, 7), (0, 7, 5, 2, 0)])
def test_random_site_order(layout, d, n_syn, R, sweeps):
    """Algs. 2-3 as printed: each step picks a generator uniformly at random
    and E_min is tracked after every step.  Every chain (E, E_min, stop step,
    final state) and the recovery (the best chain's state kept at its first
    E_min) equal the oracle's random-site chains; ragged tails of 64-chain
    tasks."""
    prob = Problem(layout, d, 0.15, 5.0, n_syn, R, sweeps, sched=("paper_log", 0.9, 1.0), seed=900 + d, conv=1)
    plan = gpu_plan(prob)
    plan.set_order(X.ORDER_RANDOM_SITE)
    assert plan.info()["kernel"] == X.KERNEL_SITE
    out = run_decode(prob, plan)
    compare_decode(prob, out, prob.oracle_decode(order=O.ORDER_RANDOM_SITE))


def test_random_site_plain_graph_and_mixed():
    """The random-site order in the plain form (one launch per syndrome), in a
    captured hipGraph, and beside colour-sweep groups (rotated, and planar on
    its specialised kernel) in one call."""
    ps = Problem(0, 9, 0.2, 10.0, 9, 4, 20, seed=77)
    pc = Problem(0, 11, 0.2, 10.0, 6, 16, 20, seed=77)   # same seeds: one call decodes both
    ref_s = ps.oracle_decode(order=O.ORDER_RANDOM_SITE)
    ref_c = pc.oracle_decode()
    plan_s = gpu_plan(ps)
    plan_s.set_order(X.ORDER_RANDOM_SITE)
    compare_decode(ps, run_decode(ps, plan_s, flags=X.FLAG_PLAIN), ref_s)
    plan_c = gpu_plan(pc)
    # and a planar group on its kernel specialised to d (paper set-up, N_SA = 10)
    pp = Problem(1, 7, 0.15, 5.0, 7, 10, 20, sched=("paper_log", 0.9, 1.0), seed=77, conv=1)
    ref_p = pp.oracle_decode()
    plan_p = gpu_plan(pp)
    assert plan_p.info()["kernel"] == X.KERNEL_ROWS
    gs_, os_ = D.make_group(plan_s, ps.n_rep, to_dev(ps.uid.view(np.int32)), syn=to_dev(ps.syn), want_chains=True)
    gc_, oc_ = D.make_group(plan_c, pc.n_rep, to_dev(pc.uid.view(np.int32)), syn=to_dev(pc.syn), want_chains=True)
    gp_, op_ = D.make_group(plan_p, pp.n_rep, to_dev(pp.uid.view(np.int32)), syn=to_dev(pp.syn), want_chains=True)
    G = D.Graph([gs_, gc_, gp_], ps.greedy_seed, ps.anneal_seed)
    for _ in range(3):
        G.launch()
        G.stream.synchronize()
        torch.cuda.synchronize()
        compare_decode(ps, os_, ref_s)
        compare_decode(pc, oc_, ref_c)
        compare_decode(pp, op_, ref_p)
    with pytest.raises(X.XzzxError):
        plan_s.set_order(7)
    srv = D.Server(max_slots=8, max_rep=4, max_qubits=81)
    with pytest.raises(X.XzzxError) as e:
        srv.submit(plan_s, ps.syn[0], 0, 4)
    assert e.value.rc == X.XZZX_EINVAL
    srv.close()


@pytest.mark.parametrize("layout,d,n_syn,R,K,sweeps", [(0, 3, 40, 4, 4, 30), (0, 11, 9, 8, 2, 20),
                                                       (0, 11, 5, 16, 16, 10), (1, 9, 7, 10, 1, 25),
                                                       (1, 7, 6, 8, 8, 15), (0, 21, 2, 4, 4, 6), (0, 5, 3, 2, 2, 0),
                                                       (0, 3, 9, 16, 4, 30), (0, 7, 5, 16, 1, 20),
                                                       (0, 13, 4, 32, 8, 12), (0, 15, 3, 16, 2, 8),
                                                       (0, 9, 3, 16, 4, 0), (1, 3, 11, 4, 2, 30),
                                                       (1, 15, 3, 8, 4, 6), (1, 11, 5, 12, 4, 10),
                                                       (0, 17, 2, 16, 4, 6), (0, 23, 2, 16, 2, 4),
                                                       (0, 31, 1, 16, 16, 3), (1, 13, 3, 8, 2, 6),
                                                       (1, 5, 6, 4, 2, 20)])
def test_replica_exchange_ladders(layout, d, n_syn, R, K, sweeps):
    """Replica exchange: ladders of K levels from beta 0.4 to 1.6 (replicas
    of a ladder share one greedy reference); every chain (E, E_min, stop,
    final state), the coset minima and the recovery (the best chain's state
    kept at its first E_min) equal the oracle's ladders, for ladders of one
    to sixteen levels, both layouts, ragged tails and zero sweeps.  Rotated
    lattices with 4R a multiple of 64 (d <= 31) and every planar d <= 15 run
    on the packed-row kernels specialised to d, the rest on the generic
    ladder kernel."""
    prob = Problem(layout, d, 0.15, 5.0, n_syn, R, sweeps, seed=1200 + d + K, conv=1 if layout else 0)
    plan = gpu_plan(prob)
    plan.set_ladder(K, 0.4, 1.6)
    assert plan.info()["kernel"] == X.KERNEL_LADDER
    out = run_decode(prob, plan)
    compare_decode(prob, out, prob.oracle_decode(order=O.ORDER_LADDER, ladder=(K, 0.4, 1.6)))


def test_replica_exchange_plain_graph_and_errors():
    """Ladders in the plain form, in a captured hipGraph beside an annealing
    group, and their argument checks."""
    pl_ = Problem(0, 9, 0.2, 10.0, 5, 8, 12, seed=88)
    pr = Problem(0, 9, 0.2, 10.0, 3, 16, 12, seed=88)     # the rotated kernel specialised to d = 9
    pp = Problem(1, 5, 0.2, 10.0, 3, 6, 12, seed=88, conv=1)   # the planar kernel specialised to d = 5
    pa = Problem(0, 11, 0.2, 10.0, 4, 16, 12, seed=88)
    ladders = [pl_, pr, pp]
    refs = [p_.oracle_decode(order=O.ORDER_LADDER, ladder=(2 if p_ is pp else 4, 0.3, 2.0)) for p_ in ladders]
    ref_a = pa.oracle_decode()
    plans = []
    for p_, ref in zip(ladders, refs):
        plan = gpu_plan(p_)
        plan.set_ladder(2 if p_ is pp else 4, 0.3, 2.0)
        compare_decode(p_, run_decode(p_, plan, flags=X.FLAG_PLAIN), ref)
        plans.append(plan)
    plan_l = plans[0]
    plan_a = gpu_plan(pa)
    made = [D.make_group(plan, p_.n_rep, to_dev(p_.uid.view(np.int32)), syn=to_dev(p_.syn), want_chains=True)
            for plan, p_ in zip(plans + [plan_a], ladders + [pa])]
    G = D.Graph([g for g, _ in made], pl_.greedy_seed, pl_.anneal_seed)
    for _ in range(3):
        G.launch()
        G.stream.synchronize()
        torch.cuda.synchronize()
        for (_, o), p_, ref in zip(made, ladders + [pa], refs + [ref_a]):
            compare_decode(p_, o, ref)
    with pytest.raises(X.XzzxError):
        plan_l.set_ladder(3, 0.3, 2.0)
    with pytest.raises(X.XzzxError):
        plan_l.set_order(X.ORDER_RANDOM_SITE)
    with pytest.raises(X.XzzxError) as e:
        D.decode(plan_l, to_dev(pl_.syn), to_dev(pl_.uid.view(np.int32)), 6, 1, 2)
    assert e.value.rc == X.XZZX_EINVAL
    srv = D.Server(max_slots=8, max_rep=8, max_qubits=81)
    with pytest.raises(X.XzzxError):
        srv.submit(plan_l, pl_.syn[0], 0, 8)
    srv.close()
    plan_l.set_ladder(0)
    assert plan_l.info()["kernel"] != X.KERNEL_LADDER


@pytest.mark.parametrize("d", [9, 25])
def test_all_lane_counts_agree(d):
    """Lanes per chain (chains per wavefront) is a result-invariant knob."""
    prob = Problem(0, d, 0.2, 10.0, 5, 16, 12, seed=50 + d)
    ref = prob.oracle_decode()
    for lanes in (1, 2, 4, 8, 16, 32, 64):
        plan = gpu_plan(prob)
        try:
            plan.set_lanes(lanes)
        except X.XzzxError as e:
            assert e.rc == X.XZZX_ERANGE   # too many chains for LDS at this d
            continue
        out = run_decode(prob, plan)
        compare_decode(prob, out, ref)


@pytest.mark.parametrize("d", [3, 11, 13, 15, 21, 29])
def test_row_and_byte_kernels_agree(d):
    """The packed-row kernel (1 or 2 words per row) and the byte-state kernel
    give identical chains; both match the oracle."""
    prob = Problem(0, d, 0.2, 10.0, 3 if d > 15 else 7, 5, 10 if d > 15 else 30, seed=300 + d)
    ref = prob.oracle_decode()
    for kernel in (X.KERNEL_ROWS, X.KERNEL_BYTES):
        plan = gpu_plan(prob)
        plan.set_kernel(kernel)
        compare_decode(prob, run_decode(prob, plan), ref)
    with pytest.raises(X.XzzxError):
        gpu_plan(Problem(1, 17, 0.2, 10.0, 1, 1, 1)).set_kernel(X.KERNEL_ROWS)


@pytest.mark.parametrize("d,n_syn,R,sweeps", [(3, 60, 3, 40), (5, 20, 10, 100), (7, 9, 7, 30), (9, 24, 10, 100),
                                              (11, 5, 10, 20), (13, 3, 12, 10), (15, 3, 16, 12)])
def test_planar_packed_rows(d, n_syn, R, sweeps):
    """Planar lattices on the packed-row kernels: turned by 45 degrees, each
    generator covers a 2 x 2 block of a diamond of rows (one word per row up
    to d = 7, two up to d = 15), in registers for the kernel specialised to
    d, in LDS for the generic one.  The paper's set-up (1:eta:1, log
    schedule; N_SA = 10 gives tasks of 64 chains spanning syndromes); both,
    the byte-state kernel and the oracle agree chain by chain."""
    prob = Problem(1, d, 0.15, 5.0, n_syn, R, sweeps, sched=("paper_log", 0.9, 1.0), seed=600 + d, conv=1)
    ref = prob.oracle_decode()
    for kernel in (X.KERNEL_ROWS, X.KERNEL_ROWS_GENERIC, X.KERNEL_BYTES):
        plan = gpu_plan(prob)
        plan.set_kernel(kernel)
        assert plan.info()["kernel"] == kernel
        compare_decode(prob, run_decode(prob, plan, want_final=True), ref)
        compare_decode(prob, run_decode(prob, plan, flags=X.FLAG_PLAIN), ref)


@pytest.mark.parametrize("d", list(range(3, 32, 2)))
def test_specialised_row_kernel(d):
    """The packed-row kernel specialised to d (registers for rows, compile-time
    schedule) runs when every 64-chain task lies in one syndrome; its chains,
    final states and results equal the generic packed-row kernel's (d <= 29),
    the byte-state kernel's and the oracle's, in the persistent and plain
    forms.  Rows take one word up to d = 15 and two words up to d = 31."""
    R = 16 if d > 9 else 32
    prob = Problem(0, d, 0.2, 10.0, 3 if d <= 21 else 2, R, 24 if d <= 21 else 12, seed=700 + d)
    ref = prob.oracle_decode()
    plan = gpu_plan(prob)
    assert plan.info()["kernel"] == X.KERNEL_ROWS
    compare_decode(prob, run_decode(prob, plan), ref)
    compare_decode(prob, run_decode(prob, plan, flags=X.FLAG_PLAIN), ref)
    if d <= 29:
        plan.set_kernel(X.KERNEL_ROWS_GENERIC)
        assert plan.info()["kernel"] == X.KERNEL_ROWS_GENERIC
        compare_decode(prob, run_decode(prob, plan), ref)
    else:
        with pytest.raises(X.XzzxError):
            plan.set_kernel(X.KERNEL_ROWS_GENERIC)
    plan.set_kernel(X.KERNEL_BYTES)
    compare_decode(prob, run_decode(prob, plan), ref)
    plan.set_kernel(X.KERNEL_AUTO)
    assert plan.info()["kernel"] == X.KERNEL_ROWS


@pytest.mark.parametrize("d,sweeps", [(7, 64), (7, 65), (7, 300), (7, 2100), (15, 300), (19, 300), (31, 300)])
def test_replay_from_checkpoints(d, sweeps):
    """Groups on the specialised kernel keep a state checkpoint every 64
    sweeps, or at most 32 evenly spaced; each syndrome's recovery is
    replayed from the last checkpoint before its E_min phase (64 sweeps:
    none; 65: one, at the start of the last sweep; 300: four; 2100: 31,
    66 sweeps apart; d = 15 stores one word per row, d = 19 and d = 31
    two)."""
    prob = Problem(0, d, 0.2, 10.0, 4 if d < 15 else 2, 16, sweeps, seed=800 + sweeps + d)
    plan = gpu_plan(prob)
    assert plan.info()["kernel"] == X.KERNEL_ROWS
    compare_decode(prob, run_decode(prob, plan), prob.oracle_decode())


def test_specialised_kernel_not_applicable():
    """Planar lattices run on the kernel specialised to d (odd d <= 15) by
    default, on the generic packed-row kernel when asked, and on the
    byte-state kernel beyond d = 15; at rotated d = 31 a replica count that
    splits 64-chain tasks over syndromes runs on the byte-state kernel (there
    is no generic packed-row kernel at d = 31)."""
    plan = gpu_plan(Problem(1, 5, 0.2, 10.0, 1, 1, 1))
    assert plan.info()["kernel"] == X.KERNEL_ROWS
    plan.set_kernel(X.KERNEL_ROWS_GENERIC)
    assert plan.info()["kernel"] == X.KERNEL_ROWS_GENERIC
    plan.set_kernel(X.KERNEL_AUTO)
    assert plan.info()["kernel"] == X.KERNEL_ROWS
    assert gpu_plan(Problem(1, 17, 0.2, 10.0, 1, 1, 1)).info()["kernel"] == X.KERNEL_BYTES
    prob = Problem(0, 31, 0.2, 10.0, 3, 5, 6, seed=931)
    compare_decode(prob, run_decode(prob, gpu_plan(prob)), prob.oracle_decode())


def test_autotuned_plan_matches_oracle():
    """The autotuner only chooses among result-invariant launch knobs."""
    for d, R in [(9, 8), (25, 4)]:
        prob = Problem(0, d, 0.2, 10.0, 4, R, 25, seed=400 + d)
        plan = gpu_plan(prob)
        tuned = plan.autotune(R, n_syn=64, probe_sweeps=10)
        print(f"[autotune] d={d}: {tuned}", flush=True)
        assert tuned["times_ms"]
        compare_decode(prob, run_decode(prob, plan), prob.oracle_decode())


def test_plain_form_matches_persistent():
    prob = Problem(0, 7, 0.15, 10.0, 9, 4, 40, seed=77)
    ref = prob.oracle_decode()
    for kernel in (X.KERNEL_ROWS, X.KERNEL_BYTES):
        plan = gpu_plan(prob)
        plan.set_kernel(kernel)
        compare_decode(prob, run_decode(prob, plan, flags=X.FLAG_PLAIN), ref)
        compare_decode(prob, run_decode(prob, plan, flags=0), ref)


@pytest.mark.parametrize("R", [4, 16])
def test_mixed_distances_one_launch(R):
    """Uneven distances in one persistent launch (groups of d = 5..21).  With
    R = 16 the groups of d <= 13 run on the specialised packed-row kernels and
    the others on the generic one, all in one decode call."""
    probs = [Problem(0, d, 0.18, 10.0, n, R, 30, seed=200 + d) for d, n in [(5, 7), (9, 5), (13, 3), (17, 2), (21, 2)]]
    groups, outs = [], []
    for prob in probs:
        plan = gpu_plan(prob)
        g, o = D.make_group(plan, prob.n_rep, to_dev(prob.uid.view(np.int32)), syn=to_dev(prob.syn),
                            want_chains=True, want_final=True)
        groups.append(g)
        outs.append(o)
    # one seed pair for the whole launch
    for p in probs:
        p.greedy_seed, p.anneal_seed = probs[0].greedy_seed, probs[0].anneal_seed
    D.decode_groups(groups, probs[0].greedy_seed, probs[0].anneal_seed)
    torch.cuda.synchronize()
    for prob, o in zip(probs, outs):
        compare_decode(prob, o, prob.oracle_decode())


def test_edge_cases():
    # no sweeps: E_min is the initial energy of each chain
    prob = Problem(0, 5, 0.2, 10.0, 6, 3, 0, seed=5)
    compare_decode(prob, run_decode(prob), prob.oracle_decode())
    # beta = 0 everywhere: every move accepted
    prob = Problem(0, 5, 0.2, 10.0, 4, 2, 9, seed=6, beta=np.zeros(9))
    compare_decode(prob, run_decode(prob), prob.oracle_decode())
    # very cold: only dE <= 0 moves
    prob = Problem(0, 7, 0.2, 10.0, 4, 2, 9, seed=7, beta=np.full(9, 1e6))
    compare_decode(prob, run_decode(prob), prob.oracle_decode())
    # the same extremes on the specialised packed-row kernel
    for beta in (np.zeros(7), np.full(7, 1e6)):
        prob = Problem(0, 7, 0.2, 10.0, 2, 16, 7, seed=17, beta=beta)
        compare_decode(prob, run_decode(prob), prob.oracle_decode())
    # single chain group tail: n_syn * 4R not a multiple of the chains per wave
    prob = Problem(0, 11, 0.2, 100.0, 3, 3, 20, seed=8)
    compare_decode(prob, run_decode(prob), prob.oracle_decode())
    # empty batch is a no-op
    prob = Problem(0, 5, 0.2, 10.0, 0, 2, 5, seed=9)
    plan = gpu_plan(prob)
    out = D.decode(plan, torch.zeros((0, prob.olat.nstab), dtype=torch.uint8, device="cuda"),
                   torch.zeros(0, dtype=torch.int32, device="cuda"), 2, 1, 2)
    torch.cuda.synchronize()
    assert out.e_best.numel() == 0


def test_anneal_from_given_references():
    """xzzx_anneal: annealing from caller-supplied references (here the
    oracle's own greedy output) without the greedy stage."""
    prob = Problem(0, 9, 0.15, 10.0, 6, 4, 30, seed=31)
    ref = prob.oracle_decode()
    plan = gpu_plan(prob)
    refs = to_dev(np.stack([r["refs"] for r in ref]))
    qcls = to_dev(np.stack([r["qcls"] for r in ref]).astype(np.uint8))
    g, o = D.make_group(plan, prob.n_rep, to_dev(prob.uid.view(np.int32)), refs=refs, qcls=qcls,
                        want_chains=True, want_final=True)
    D.anneal_groups([g], prob.anneal_seed)
    torch.cuda.synchronize()
    compare_decode(prob, o, ref)


def test_graph_replays_match_eager():
    prob = Problem(0, 9, 0.2, 10.0, 10, 8, 25, seed=44)
    ref = prob.oracle_decode()
    plan = gpu_plan(prob)
    syn = to_dev(prob.syn)
    uid = to_dev(prob.uid.view(np.int32))
    g, o = D.make_group(plan, prob.n_rep, uid, syn=syn, want_chains=True, want_final=True)
    graph = D.Graph([g], prob.greedy_seed, prob.anneal_seed)
    for rep in range(3):
        for t in (o.e_best, o.recovery, o.chain_emin, o.chain_final):
            t.fill_(0x55 if t.dtype == torch.uint8 else -7)
        graph.launch()
        graph.stream.synchronize()
        compare_decode(prob, o, ref)
        # eager work in between replays
        out2 = run_decode(prob, plan)
        compare_decode(prob, out2, ref)


def test_bad_arguments_raise():
    prob = Problem(0, 5, 0.2, 10.0, 4, 2, 5, seed=3)
    plan = gpu_plan(prob)
    with pytest.raises(X.XzzxError):
        plan.set_lanes(3)
    g, o = D.make_group(plan, 2, to_dev(prob.uid.view(np.int32)), syn=to_dev(prob.syn))
    tiny = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(X.XzzxError) as e:
        D.decode_groups([g], 1, 2, ws=tiny)
    assert e.value.rc == X.XZZX_ENOMEM
