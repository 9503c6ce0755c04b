"""Statistical trends of the paper's own set-up, decoded on the GPU (Sec. V):
planar layout, p_x:p_y:p_z = 1:eta:1, log schedule 0.9 beta_N -> beta_N
(Eqs. 23-24).  Every setting decodes the same seeded syndromes, so two
settings are compared pair by pair: `better` counts syndromes only the
setting the paper finds better decodes, `worse` the reverse, and the sign
test z = (better - worse) / sqrt(better + worse) must exceed 4.

* P_L falls as N_SA grows (Figs. 6-8);
* SA with N_SA >= 2 beats the greedy-matching decoder of Alg. 5 (Sec. V.B);
* greedy (different) references beat greedy (same), which beat the boundary
  construction, at fixed N_beta (Sec. V.C, Figs. 9-11).

Logical failure is judged by the oracle's class of error * recovery, so the
check is independent of the HIP path."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_17837_amd import _lib as X
from paper_2509_17837_amd import decoder as D
from paper_2509_17837_amd import inputs

pytestmark = pytest.mark.gpu

D_, P_, ETA, N = 9, 0.15, 5.0, 4000
Z_MIN = 4.0


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    lat = D.Lattice(X.PLANAR, D_)
    olat = O.Lattice(O.PLANAR, D_)
    w, wg = D.weights(P_, D.noise(P_, ETA, X.BIAS_PAPER))
    err = inputs.sample_errors(N, lat.nq, inputs.channel(P_, ETA, 1), 9090, stream=5)
    uid = torch.from_numpy(inputs.sample_uids(N).view(np.int32)).cuda()
    syn = torch.from_numpy(np.stack([olat.syndrome(e) for e in err])).cuda()
    print(f"[trends] planar d={D_} p={P_} eta={ETA} syndromes={N}", flush=True)

    def plan(n_beta):
        return D.Plan(lat, w, wg, D.schedule(X.SCHED_PAPER_LOG, 0.9, 1.0, n_beta))

    def fails(recovery):
        rec = recovery.cpu().numpy()
        return np.array([olat.cls(err[i], rec[i]) != 0 for i in range(N)])

    return dict(plan=plan, fails=fails, syn=syn, uid=uid)


def sign_z(f_good, f_bad):
    better = int(np.count_nonzero(~f_good & f_bad))
    worse = int(np.count_nonzero(f_good & ~f_bad))
    return (better - worse) / np.sqrt(max(better + worse, 1)), better, worse


def decode_fails(s, plan, n_sa, mode=X.GREEDY_RANDOM):
    o = D.decode(plan, s["syn"], s["uid"], n_sa, 11, 22, greedy_mode=mode)
    torch.cuda.synchronize()
    return s["fails"](o.recovery)


def test_p_l_falls_with_n_sa_and_beats_greedy(setup):
    s = setup
    plan = s["plan"](100)
    f = {k: decode_fails(s, plan, k) for k in (1, 2, 3, 10)}
    refs, _ = D.greedy_init(plan, s["syn"], s["uid"], 1, 11, X.GREEDY_SAME)
    f_greedy = s["fails"](refs[:, 0])
    print("[trends] P_L greedy %.4f, " % f_greedy.mean() +
          ", ".join(f"N_SA={k}: {v.mean():.4f}" for k, v in f.items()), flush=True)
    for a, b in ((1, 3), (3, 10)):
        z, better, worse = sign_z(f[b], f[a])
        assert z > Z_MIN, f"N_SA {a} -> {b}: better {better}, worse {worse}"
    for k in (2, 3, 10):
        z, better, worse = sign_z(f[k], f_greedy)
        assert z > Z_MIN, f"N_SA {k} vs greedy: better {better}, worse {worse}"


@pytest.mark.parametrize("n_beta", [0, 10, 100])
def test_reference_construction_ranking(setup, n_beta):
    s = setup
    plan = s["plan"](n_beta)
    f = {m: decode_fails(s, plan, 10, m) for m in (X.GREEDY_RANDOM, X.GREEDY_SAME, X.GREEDY_BOUNDARY)}
    print(f"[trends] N_beta={n_beta}: P_L different {f[X.GREEDY_RANDOM].mean():.4f}, "
          f"same {f[X.GREEDY_SAME].mean():.4f}, boundary {f[X.GREEDY_BOUNDARY].mean():.4f}", flush=True)
    z, better, worse = sign_z(f[X.GREEDY_RANDOM], f[X.GREEDY_SAME])
    assert z > Z_MIN, f"different vs same: better {better}, worse {worse}"
    z, better, worse = sign_z(f[X.GREEDY_SAME], f[X.GREEDY_BOUNDARY])
    assert z > Z_MIN, f"same vs boundary: better {better}, worse {worse}"
