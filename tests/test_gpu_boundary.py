"""The C ABI's stream and argument contract on the GPU: the anneal-only entry
point checks and classifies caller references; calls on different streams and
threads (a graph capture, a serving loop, eager decodes) share no internal
stream and give the same results as alone; the Python face allocates for the
stream a call runs on."""
import threading

import numpy as np
import pytest
import torch

from paper_2509_17837_amd import _lib as X
from paper_2509_17837_amd import decoder as D
from tests._parity import Problem, compare_decode, gpu_plan, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    X.lib()
    torch.cuda.synchronize()


def test_anneal_checks_and_classifies_references():
    """xzzx_anneal computes each reference's class on the device (Alg. 7,
    Eqs. (35)-(36)) whatever d_qcls held, and with d_syn given rejects a
    reference whose syndrome is not S (EINVAL) before any annealing."""
    prob = Problem(0, 9, 0.15, 10.0, 6, 4, 30, seed=31)
    ref = prob.oracle_decode()
    plan = gpu_plan(prob)
    refs_np = np.stack([r["refs"] for r in ref])
    uid = to_dev(prob.uid.view(np.int32))
    syn = to_dev(prob.syn)
    print("[boundary] anneal with d_syn, wrong d_qcls", flush=True)
    qcls = torch.full((prob.n_syn, prob.n_rep), 0xEE, dtype=torch.uint8, device="cuda")
    g, o = D.make_group(plan, prob.n_rep, uid, syn=syn, refs=to_dev(refs_np), qcls=qcls, want_chains=True,
                        want_final=True)
    D.anneal_groups([g], prob.anneal_seed)
    torch.cuda.synchronize()
    compare_decode(prob, o, ref)          # qcls compared with the oracle's too
    print("[boundary] anneal without d_qcls", flush=True)
    g, o = D.make_group(plan, prob.n_rep, uid, refs=to_dev(refs_np), want_extra=False, want_chains=True)
    D.anneal_groups([g], prob.anneal_seed)
    torch.cuda.synchronize()
    assert np.array_equal(o.e_best.cpu().numpy(), [r["e_best"] for r in ref])
    assert np.array_equal(o.recovery.cpu().numpy(), np.stack([r["recovery"] for r in ref]))
    print("[boundary] anneal with a corrupted reference", flush=True)
    bad = refs_np.copy()
    bad[2, 1, 17] ^= 2                     # one X flipped: the syndrome changes
    assert not np.array_equal(prob.olat.syndrome(bad[2, 1]), prob.syn[2])
    g, o = D.make_group(plan, prob.n_rep, uid, syn=syn, refs=to_dev(bad), want_chains=True)
    with pytest.raises(X.XzzxError) as e:
        D.anneal_groups([g], prob.anneal_seed)
    assert e.value.rc == X.XZZX_EINVAL
    torch.cuda.synchronize()
    # unchecked without d_syn: the call is accepted
    g, o = D.make_group(plan, prob.n_rep, uid, refs=to_dev(bad), want_chains=True)
    D.anneal_groups([g], prob.anneal_seed)
    torch.cuda.synchronize()
    print("[boundary] checked anneal under capture is refused", flush=True)
    g, o = D.make_group(plan, prob.n_rep, uid, syn=syn, refs=to_dev(refs_np), want_chains=True)
    ws = D.workspace([g])
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side, capture_error_mode="thread_local"):
        with pytest.raises(X.XzzxError) as e:
            D.anneal_groups([g], prob.anneal_seed, ws=ws, stream=side)
    assert e.value.rc == X.XZZX_EINVAL
    torch.cuda.synchronize()


def test_decode_on_a_side_stream_while_current_stream_allocates():
    """The Python face allocates a call's outputs and workspace for the stream
    the call runs on and marks its inputs as used there, so memory churn on the
    current stream while a long decode runs elsewhere cannot reuse its
    buffers."""
    prob = Problem(0, 11, 0.2, 100.0, 48, 8, 400, seed=71)
    ref = prob.oracle_decode(chains=True)
    plan = gpu_plan(prob)
    side = torch.cuda.Stream()
    syn = to_dev(prob.syn)
    uid = to_dev(prob.uid.view(np.int32))
    torch.cuda.synchronize()
    print("[boundary] decode on a side stream", flush=True)
    out = D.decode(plan, syn, uid, prob.n_rep, prob.greedy_seed, prob.anneal_seed, want_chains=True,
                   want_final=True, stream=side)
    del syn, uid
    junk = []
    for k in range(48):
        t = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
        t.fill_(k)
        junk.append(t)
        if k % 3 == 0:
            junk.pop(0)
    side.synchronize()
    torch.cuda.synchronize()
    compare_decode(prob, out, ref)


def test_capture_serving_and_eager_calls_in_parallel():
    """A graph captured on one thread's stream, a serving loop (its own
    stream and scheduler thread) and eager multi-group decodes on a third
    stream run at the same time; each result equals the same work done
    alone."""
    a = Problem(0, 9, 0.2, 10.0, 12, 8, 60, seed=81)
    b = Problem(0, 7, 0.2, 10.0, 12, 8, 60, seed=82)
    b.greedy_seed, b.anneal_seed = a.greedy_seed, a.anneal_seed   # one decode call covers both groups
    plan_a, plan_b = gpu_plan(a), gpu_plan(b)
    ref_a, ref_b = a.oracle_decode(chains=False), b.oracle_decode(chains=False)

    def groups(stream=None):
        ga, oa = D.make_group(plan_a, a.n_rep, to_dev(a.uid.view(np.int32)), syn=to_dev(a.syn), stream=stream)
        gb, ob = D.make_group(plan_b, b.n_rep, to_dev(b.uid.view(np.int32)), syn=to_dev(b.syn), stream=stream)
        return [ga, gb], [oa, ob]

    def check(outs):
        for prob, o, ref in ((a, outs[0], ref_a), (b, outs[1], ref_b)):
            assert np.array_equal(o.e_best.cpu().numpy(), [r["e_best"] for r in ref])
            assert np.array_equal(o.recovery.cpu().numpy(), np.stack([r["recovery"] for r in ref]))

    errors = []

    def capture_thread():
        try:
            s = torch.cuda.Stream()
            for _ in range(4):
                gs, outs = groups(stream=s)
                ws = D.workspace(gs, stream=s)
                s.synchronize()
                graph = D.Graph(gs, a.greedy_seed, a.anneal_seed, stream=s, ws=ws)
                for _ in range(2):
                    graph.launch(s)
                    s.synchronize()
                    check(outs)
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    srv = D.Server(max_slots=64, max_rep=8, max_qubits=81, sweeps_per_slice=20, greedy_seed=a.greedy_seed,
                   anneal_seed=a.anneal_seed)
    print("[boundary] capture thread + server + eager decodes", flush=True)
    th = threading.Thread(target=capture_thread)
    th.start()
    tickets = [srv.submit(plan_a, a.syn[i], int(a.uid[i]), a.n_rep) for i in range(a.n_syn)]
    eager = torch.cuda.Stream()
    for _ in range(4):
        gs, outs = groups(stream=eager)
        D.decode_groups(gs, a.greedy_seed, a.anneal_seed, stream=eager)
        eager.synchronize()
        check(outs)
    th.join()
    srv.drain()
    for i, t in enumerate(tickets):
        res = srv.poll(t)
        assert res["e_best"] == ref_a[i]["e_best"] and np.array_equal(res["recovery"], ref_a[i]["recovery"])
    srv.close()
    assert not errors, errors
    torch.cuda.synchronize()
