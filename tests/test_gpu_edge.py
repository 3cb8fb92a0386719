"""Edge cases of the step on the GPU against the oracle: the smallest chain
(N = 2, both beads are ends), workgroups with a ragged tail (fewer chains than
a group holds, a wave only partly filled), zero-step calls, one-step
launches that start at odd steps (the step-pair random streams rebuild their
carry), and states with many springs on one bead (the force gather adds them
in slot order, over every width of the beads' slot masks)."""
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


def _compare_run(lengths, precision, steps, seed, kappa=None, launch=1, state=None, mapping=None):
    e = _ens(np.array(lengths), precision=precision, seed=seed, corr_levels=0).init()
    o = oracle.Ensemble(lengths, seed=seed).init()
    if mapping is not None:
        e.set_mapping(*mapping)
    if state is not None:
        R, A, S = state
        e.write_state(R, A, S)
        o.R[:] = R
        o.A[:] = A
        o.S[:] = S
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


def _crowded_state(lengths, rng):
    """Random-walk chains whose slots pile onto few beads: chains 0, 3, ...
    hold every slot on bead 5 (or the last bead of a shorter chain), chains
    1, 4, ... alternate their slots between the two ends, and the others put
    about half of their slots on bead 1 and the rest anywhere or empty."""
    R, A, S = [], [], []
    for c, n in enumerate(lengths):
        r = np.cumsum(rng.normal(0.0, np.sqrt(1.0 / 3.0), (n, 3)), axis=0)
        if c % 3 == 0:
            s = np.full(n, min(5, n - 1))
        elif c % 3 == 1:
            s = np.where(np.arange(n) % 2 == 0, 0, n - 1)
        else:
            s = np.where(rng.random(n) < 0.5, 1, rng.integers(-1, n, n))
        a = r[np.maximum(s, 0)] + rng.normal(0.0, np.sqrt(0.5 / 3.0), (n, 3))
        a[s < 0] = 0.0
        R.append(r)
        A.append(a)
        S.append(s)
    return np.concatenate(R), np.concatenate(A), np.concatenate(S).astype(np.int32)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N,W,B", [(8, 8, 1), (32, 32, 1), (32, 16, 2), (32, 64, 1), (64, 64, 1), (64, 32, 2),
                                   (128, 64, 2)])
def test_crowded_beads_gather_in_slot_order(precision, N, W, B):
    """Up to N springs on one bead, in every mask width (one, two and four
    32-bit words per bead) and with two beads per lane; launches of four
    steps, so the masks are rebuilt inside a launch."""
    lengths = [N] * 6
    state = _crowded_state(lengths, np.random.default_rng(1000 + N + W + B))
    worst = _compare_run(lengths, precision, 8, seed=26, launch=4, state=state, mapping=(N, N, W, B))
    print(precision, N, W, B, "crowded worst", worst)


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
