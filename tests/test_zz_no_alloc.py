"""xzzx_decode_noalloc: the decode with the library's static per-device
workspace equals xzzx_decode with a caller workspace, on two calls in a row
(the second smaller, so it runs over the first call's leftovers), and rejects
groups whose workspace exceeds the static array."""
import numpy as np
import pytest
import torch

from paper_2509_17837_amd import _lib as X
from paper_2509_17837_amd import decoder as D
from tests._parity import Problem, compare_decode, gpu_plan, to_dev

pytestmark = pytest.mark.gpu

FIELDS = ("e_best", "cls", "recovery", "paper_recovery", "e_cls", "best_chain", "refs", "qcls", "chain_emin",
          "chain_stop", "chain_e", "chain_final")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    X.lib()
    torch.cuda.synchronize()


def _groups(probs, plans):
    gs, outs = [], []
    for prob, plan in zip(probs, plans):
        g, o = D.make_group(plan, prob.n_rep, to_dev(prob.uid.view(np.int32)), syn=to_dev(prob.syn),
                            want_chains=True, want_final=True)
        gs.append(g)
        outs.append(o)
    return gs, outs


def test_no_alloc_matches_decode():
    calls = [
        # mixed distances; d = 11 with 64-chain tasks runs the specialised
        # kernel and its checkpoints (300 sweeps)
        [Problem(0, 11, 0.2, 100.0, 24, 16, 300, seed=91), Problem(0, 7, 0.15, 10.0, 13, 5, 80, seed=92),
         Problem(1, 5, 0.1, 5.0, 9, 3, 40, seed=93, conv=1)],
        # second call, smaller: one group
        [Problem(0, 9, 0.2, 10.0, 5, 4, 50, seed=94)],
    ]
    for k, probs in enumerate(calls):
        plans = [gpu_plan(p) for p in probs]
        gs_ref, outs_ref = _groups(probs, plans)
        gs, outs = _groups(probs, plans)
        nbytes = D.workspace(gs).numel()
        assert nbytes <= X.NOALLOC_SCRATCH_BYTES
        print(f"[no-alloc] call {k}: {len(probs)} groups, workspace {nbytes} bytes", flush=True)
        for o in outs:
            for t in (o.e_best, o.recovery, o.chain_emin, o.chain_final):
                t.fill_(0x55 if t.dtype == torch.uint8 else -7)
        torch.cuda.synchronize()
        ws = D.decode_groups(gs_ref, 0x5EED, 0xA11E)
        D.decode_groups_noalloc(gs, 0x5EED, 0xA11E)
        torch.cuda.synchronize()
        del ws
        for prob, o, r in zip(probs, outs, outs_ref):
            for f in FIELDS:
                a, b = getattr(o, f), getattr(r, f)
                assert torch.equal(a, b), f"call {k} d={prob.d}: {f}"
        # and the oracle on two syndromes of the first group
        prob = probs[0]
        prob.greedy_seed, prob.anneal_seed = 0x5EED, 0xA11E
        ref = prob.oracle_decode(idx=[0, prob.n_syn - 1])
        sub = type(outs[0])(**{f: (getattr(outs[0], f)[[0, prob.n_syn - 1]] if getattr(outs[0], f) is not None
                                   else None) for f in FIELDS})
        compare_decode(prob, sub, ref)


def test_no_alloc_rejects_oversized_groups():
    prob = Problem(0, 11, 0.2, 100.0, 0, 32, 2000, seed=95)
    plan = gpu_plan(prob)
    n = 4096
    uid = torch.zeros(n, dtype=torch.int32, device="cuda")
    syn = torch.zeros((n, prob.olat.nstab), dtype=torch.uint8, device="cuda")
    g, o = D.make_group(plan, 32, uid, syn=syn)
    assert D.workspace([g]).numel() > X.NOALLOC_SCRATCH_BYTES
    with pytest.raises(X.XzzxError) as e:
        D.decode_groups_noalloc([g], 1, 2)
    assert e.value.rc == X.XZZX_ERANGE
