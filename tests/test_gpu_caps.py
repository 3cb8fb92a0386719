"""Step-by-step parity where the caps of the Sec. 3.1 step map bind: the hop
probabilities min{(dt/zeta_s)[1 - tanh(...)], 1/2}, the construction
probability min{dt/(zeta_s N_0 K), 1/2} per attempt and end, and the
destruction probability min{(dt/zeta_s)(delta_{S,1} + delta_{S,N}), 1}.

At the paper's dt/zeta_s = 0.1 none of them binds.  Here:
  * dt/zeta_s = 0.5 (zeta_s = 0.02): a hop probability is capped whenever the
    energy difference is negative;
  * dt/zeta_s = 4 with N_0 = 1 (zeta_s = 0.0025): every hop probability,
    construction at K <= 8 and destruction (probability 1) are capped.
The library accepts both with a warning.  Bars as in the other stepwise
tests: FP64 1e-12 with identical decisions, FP32 1e-5 with margin-checked
ties.  The oracle's own events confirm that the caps were exercised.
"""
import numpy as np
import pytest

import oracle

from _lockstep import lockstep

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EV_HOP_UP, EV_HOP_DOWN, EV_DESTROY, EV_CREATE_FIRST, EV_CREATE_LAST = 1, 2, 4, 8, 16


def _run(precision, M, N, steps, zeta_s, n0, kappa=None, rule=0, seed=21):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1106_2899_amd.ensemble import Ensemble
    with pytest.warns(UserWarning, match="dt/zeta_s"):
        e = Ensemble(N, M, precision=precision, seed=seed, corr_levels=0, zeta_s=zeta_s, n0=n0,
                     construct_rule=rule).init()
    o = oracle.Ensemble([N] * M, seed=seed, zeta_s=zeta_s, n0=n0, construct_rule=rule).init()
    kap = None if kappa is None else np.asarray(kappa, dtype=np.float64).reshape(1, 9)
    kchain = None if kap is None else np.repeat(kap, M, axis=0)
    tally = {"hop_decisions": 0, "hop_capped": 0, "destroyed": 0, "created": 0, "attempts": 0}

    def on_step(t, o, ev, pre):
        S0 = pre[2]
        ev = ev.reshape(-1)
        tally["destroyed"] += int(((ev & EV_DESTROY) != 0).sum())
        tally["created"] += int(((ev & (EV_CREATE_FIRST | EV_CREATE_LAST)) != 0).sum())
        tally["attempts"] += int((S0 < 0).sum())
        if t % 5:
            return
        # hop probabilities of the springs that survive the step, from the
        # post-move positions (unchanged by hops and reconstruction)
        for k in range(M):
            r = o.R[k * N:(k + 1) * N]
            for j in range(N):
                q = k * N + j
                if S0[q] < 0 or o.S[q] < 0:
                    continue
                for direction in (+1, -1):
                    i = int(S0[q])
                    if (direction > 0 and i == N - 1) or (direction < 0 and i == 0):
                        continue
                    p = oracle.hop_prob(r, o.A[q], i, direction, dt=0.01, ns=0.5, zeta_s=zeta_s)
                    tally["hop_decisions"] += 1
                    tally["hop_capped"] += int(p == 0.5)

    st = lockstep(e, o, steps, kappa_elem=kap, kappa_chain=kchain, tol=1e-12 if precision == "fp64" else 1e-5,
                  fp64=precision == "fp64", on_step=on_step)
    print(f"{precision} {M}x{N} dt/zeta_s = {0.01 / zeta_s:g}, N0 = {n0}: worst {st['worst']:.2e}, "
          f"ties {st['ties']}, {tally}")
    return st, tally


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_hop_cap_binds(precision):
    st, tally = _run(precision, 64, 16, 300, zeta_s=0.02, n0=4.0, kappa=[[0, 0.2, 0], [0, 0, 0], [0, 0, 0]])
    assert tally["hop_capped"] > 0.1 * tally["hop_decisions"]


@pytest.mark.parametrize("rule", [0, 1], ids=["K=C-Z", "K=1"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_cap_binds(precision, rule):
    st, tally = _run(precision, 64, 12, 300, zeta_s=0.0025, n0=1.0, kappa=[[0, 0.5, 0], [0, 0, 0], [0, 0, 0]],
                     rule=rule)
    assert tally["hop_capped"] > 0.5 * tally["hop_decisions"]
    # destruction probability min(4 (delta_S1 + delta_SN), 1) = 1: every spring
    # on an end after the hop goes, so destructions are frequent
    assert tally["destroyed"] > 0.05 * tally["hop_decisions"]
    if rule == 0:
        # p = min(4 / K, 1/2) = 1/2 per end for K <= 8 (2p = 1: the attempt
        # always creates); K = 12 - Z is at most 8 once Z >= 4
        assert tally["created"] > 0.7 * tally["attempts"]
