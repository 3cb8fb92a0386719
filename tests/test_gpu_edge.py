"""Edge cases of the step on the GPU against the oracle: the smallest chain
(N = 2, both beads are ends), workgroups with a ragged tail (fewer chains than
a group holds, a wave only partly filled), zero-step calls, and one-step
launches that start at odd steps (the step-pair random streams rebuild their
carry)."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCALE = 0.58
TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _ens(N, M=None, **kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1106_2899_amd.ensemble import Ensemble
    return Ensemble(N, M, **kw)


def _bonds_offsets(R, A, S, lengths):
    """Bond vectors and anchor offsets d_j = R_{S_j} - A_j (0 for empty slots)."""
    b, d, off = [], [], 0
    for n in lengths:
        r, a, s = R[off:off + n], A[off:off + n], S[off:off + n]
        b.append(r[1:] - r[:-1])
        d.append(np.where((s >= 0)[:, None], r[np.maximum(s, 0)] - a, 0.0))
        off += n
    return np.concatenate(b), np.concatenate(d)


def _compare_run(lengths, precision, steps, seed, kappa=None, launch=1):
    e = _ens(np.array(lengths), precision=precision, seed=seed, corr_levels=0).init()
    o = oracle.Ensemble(lengths, seed=seed).init()
    kap = None if kappa is None else np.asarray(kappa)
    worst = 0.0
    for t in range(0, steps, launch):
        e.step(launch, kap)
        for _ in range(launch):
            o.step(kap)
        R, A, S = (x.cpu().numpy() for x in e.state())
        assert np.array_equal(S, o.S), f"slot state differs after step {t + launch}"
        bg, dg = _bonds_offsets(R, A, S, lengths)
        bo, do = _bonds_offsets(o.R, o.A, o.S, lengths)
        err = max((np.abs(bg - bo) / np.maximum(np.abs(bo), SCALE)).max(),
                  (np.abs(dg - do) / np.maximum(np.abs(do), SCALE)).max())
        worst = max(worst, err)
        assert err <= TOL[precision], (t, err)
    return worst


def test_single_two_bead_chain_fp64():
    worst = _compare_run([2], "fp64", 400, seed=23)
    print("N=2 single chain fp64 worst", worst)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ragged_groups_and_partly_filled_waves(precision):
    """5 chains of N = 128 (one per wave, four per group: the second group has
    one) beside 7 chains of N = 8 (eight per wave: one wave partly filled)."""
    lengths = [128] * 5 + [8] * 7
    worst = _compare_run(lengths, precision, 150, seed=24, kappa=[[0, 0.2, 0], [0, 0, 0], [0, 0, 0]], launch=3)
    print(precision, "ragged worst", worst)


def test_zero_steps_is_a_no_op_and_odd_starts_continue_the_streams():
    kw = dict(precision="fp32", seed=25, corr_levels=4, corr_batches=2, sample_every=2)
    a = _ens(16, 40, **kw).init()
    b = _ens(16, 40, **kw).init()
    before = [x.clone() for x in a.state()]
    a.step(0)
    assert all(torch.equal(x, y) for x, y in zip(before, a.state()))
    assert a.step_count() == 0
    a.step(101)
    for n in (1, 2, 1, 3, 1, 5, 88):  # launches starting at odd and even steps
        b.step(n)
    assert a.step_count() == b.step_count() == 101
    assert all(torch.equal(x, y) for x, y in zip(a.state(), b.state()))
