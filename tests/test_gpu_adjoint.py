"""GPU pathwise adjoint (recorded window, checkpointed replay, reverse pass)
against the oracle's discrete adjoint on the same seeded inputs.  A window
recorded as one segment (checkpoint interval >= window) stores its trajectory
in the forward and is differentiated without a replay; the tests run both.

Tolerance: FP64 path 1e-9 relative to the largest gradient entry; FP32 path
1e-4 (the adjoint recursion runs in the path's precision, gradients are
accumulated in FP64).  The oracle adjoint is itself pinned to central finite
differences of its frozen-event forward (tests/test_oracle_adjoint.py).
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ens(N, M=None, **kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1106_2899_amd.ensemble import Ensemble
    return Ensemble(N, M, **kw)


def _shear(g):
    k = np.zeros((3, 3))
    k[0, 1] = g
    return k


def _oracle_grad(N, seed, T, kap, comp):
    o = oracle.Ensemble(N, seed=seed).init()
    Rt, At, St = o.run_record(T, kap)
    gk, gns = o.adjoint(Rt, At, St, kap, comp=comp)
    return np.concatenate([gk.reshape(len(N), 9), gns[:, None]], axis=1), o


def _check(got, want, rtol):
    scale = np.abs(want).max(axis=0)
    scale[scale == 0] = 1.0
    err = np.abs(got - want) / scale
    assert err.max() <= rtol, (err.max(axis=0), rtol)


@pytest.mark.parametrize("ckpt", [64, 300], ids=["checkpointed", "stored"])
@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_adjoint_matches_oracle_shear(precision, rtol, ckpt):
    N, M, T = 12, 24, 300  # segments 64, 64, 64, 64, 44, or one stored window
    kap = _shear(0.3)
    # launches of 70 steps: a stored window spans several launches
    e = _ens(N, M, precision=precision, seed=5, corr_levels=0, max_steps_per_launch=70).init()
    e.forward_record(T, ckpt, kap)
    got = e.adjoint(component=3).cpu().numpy()
    want, o = _oracle_grad([N] * M, 5, T, kap, 3)
    S_end = e.state()[2].cpu().numpy()
    assert np.array_equal(S_end, o.S)  # same events
    _check(got, want, rtol)


@pytest.mark.parametrize("ckpt", [50, 150], ids=["checkpointed", "stored"])
def test_adjoint_matches_oracle_mixed_lengths_elongation_fp64(ckpt):
    """Lengths 5..128 (one and two beads per lane): a stored window's
    destruction log is read back in the slot order it was written in."""
    N = [5, 16, 33, 70, 128, 9, 40, 100] * 3
    kap = np.diag([0.02, -0.01, -0.01])
    e = _ens(N, precision="fp64", seed=9, corr_levels=0, max_steps_per_launch=40).init()
    e.forward_record(150, ckpt, kap)
    got = e.adjoint(component=0).cpu().numpy()
    want, _ = _oracle_grad(N, 9, 150, kap, 0)
    _check(got, want, 1e-9)


@pytest.mark.parametrize("ckpt", [40, 230], ids=["checkpointed", "stored"])
def test_forward_record_advances_exactly_like_step(ckpt):
    kap = _shear(0.2)
    kw = dict(precision="fp32", seed=3, corr_levels=4, corr_batches=4, sample_every=5, max_steps_per_launch=100)
    a = _ens(20, 32, **kw).init()
    b = _ens(20, 32, **kw).init()
    a.forward_record(230, ckpt, kap)
    b.step(230, kap)
    for x, y in zip(a.state(), b.state()):
        assert torch.equal(x, y)
    assert np.array_equal(a.correlator()["G"], b.correlator()["G"])
    assert a.steps == b.steps == 230


def test_autograd_function_matches_adjoint_means():
    from paper_1106_2899_amd.adjoint import final_stress
    E, per, N = 3, 16, 10
    e = _ens(N, E * per, n_elements=E, precision="fp64", seed=11, corr_levels=0).init()
    rates = torch.tensor([0.05, 0.2, 0.6], dtype=torch.float64, requires_grad=True)
    ns = torch.tensor(0.5, dtype=torch.float64, requires_grad=True)
    shear_dir = torch.tensor([[0, 1.0, 0], [0, 0, 0], [0, 0, 0]], dtype=torch.float64)
    J = final_stress(rates, ns, e, shear_dir, 120, 40, "xy")
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64)
    (J * w).sum().backward()
    # reference: the oracle's per-chain adjoint, averaged per element
    kap = np.zeros((E * per, 3, 3))
    kap[:, 0, 1] = np.repeat(rates.detach().numpy(), per)
    o = oracle.Ensemble([N] * (E * per), seed=11).init()
    Rt, At, St = o.run_record(120, kap.reshape(-1, 9))
    gk, gns = o.adjoint(Rt, At, St, kap.reshape(-1, 9), comp=3)
    d_rate = gk[:, 0, 1].reshape(E, per).mean(axis=1)
    d_ns = gns.reshape(E, per).mean(axis=1)
    np.testing.assert_allclose(rates.grad.numpy(), w.numpy() * d_rate, rtol=1e-9)
    np.testing.assert_allclose(float(ns.grad), float((w.numpy() * d_ns).sum()), rtol=1e-9)
    np.testing.assert_allclose(J.detach().cpu().numpy(), o.stress()[:, 3].reshape(E, per).mean(axis=1), rtol=1e-10)


def test_element_reductions_of_stress_and_adjoint():
    """ssp_read_element_stress and ssp_adjoint_elements: per-element means over
    unequal elements (7, 300 and 13 chains: the middle one spans more chains
    than the reduction block has threads) against the oracle's per-chain
    stress and adjoint of the same chains, averaged per element (FP64)."""
    offs = np.array([0, 7, 307, 320])
    E, M, N, T = 3, 320, 6, 60
    rates = np.array([0.3, 0.05, 1.0])
    kap = np.zeros((E, 3, 3))
    kap[:, 0, 1] = rates
    e = _ens(N, M, n_elements=E, element_offsets=offs, precision="fp64", seed=17, corr_levels=0).init()
    e.forward_record(T, 20, kap.reshape(E, 9))
    Sel = e.element_stress().cpu().numpy()
    elem, chain = (x.cpu().numpy() for x in e.adjoint_elements(component=3))
    kchain = np.repeat(kap.reshape(E, 9), np.diff(offs), axis=0)
    o = oracle.Ensemble([N] * M, seed=17).init()
    Rt, At, St = o.run_record(T, kchain)
    gk, gns = o.adjoint(Rt, At, St, kchain, comp=3)
    so = o.stress()
    for q in range(E):
        sl = slice(offs[q], offs[q + 1])
        np.testing.assert_allclose(Sel[q], so[sl].mean(axis=0), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(elem[q, :9], gk[sl].reshape(-1, 9).mean(axis=0), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(elem[q, 9], gns[sl].mean(), rtol=1e-9, atol=1e-12)
        # the element means are the means of the per-chain values returned
        np.testing.assert_allclose(elem[q], chain[sl].mean(axis=0), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(chain[:, 9], gns, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("change", ["out_of_range", "impossible_move", "first_row", "inner_destruction"])
@pytest.mark.parametrize("ckpt", [10, 40], ids=["checkpointed", "stored"])
def test_adjoint_rejects_a_changed_recording_and_keeps_the_ensemble(ckpt, change):
    """A slot row changed after ssp_forward_record is caught where the replay
    and the adjoint read it (both kernels check a row before using it, and read
    a bad entry as an empty slot): either a state that cannot exist (100 in a
    chain of N = 8), or one no step reaches from the row before (a spring that
    appears in the middle of the chain, or vanishes more than one bead from an
    end), or a first row from which no step reaches the second (which a
    replay, starting from its checkpoint, never compares).  ssp_adjoint fails, the ensemble's own state is untouched, and a
    new recording differentiates normally."""
    from paper_1106_2899_amd._lib import SspError

    N, M, T = 8, 64, 40
    kap = _shear(0.1)
    e = _ens(N, M, precision="fp32", seed=31, corr_levels=0).init()
    e.forward_record(T, ckpt, kap)
    before = [x.clone() for x in e.state()]
    # slot rows: the first region of the recording buffer, [T + 1][N * M] int8
    off = e._rec_p - e._rec_t.data_ptr()
    rows = e._rec_t[off:off + (T + 1) * N * M].view(T + 1, N * M)
    if change == "out_of_range":
        rows[20, 3] = 100
    elif change == "impossible_move":
        r = rows.cpu().numpy().astype(np.int8)
        empty = np.flatnonzero((r[19] == -1) & (r[20] == -1) & (r[21] == -1))
        assert empty.size > 0
        rows[20, int(empty[0])] = N // 2
    elif change == "inner_destruction":
        r = rows.cpu().numpy().astype(np.int8)
        j = int(np.flatnonzero((r[19] >= 2) & (r[19] <= N - 3))[0])  # a spring away from the ends
        rows[20:, j] = 255  # int8 -1: empty
    else:
        r = rows.cpu().numpy().astype(np.int8)
        j = int(np.flatnonzero((r[0] >= 0) & (r[1] >= 0))[0])  # a spring held over step 0
        s1 = int(r[1, j])
        rows[0, j] = s1 + 3 if s1 + 3 < N else s1 - 3
    torch.cuda.synchronize()
    with pytest.raises(SspError, match="recorded slot rows"):
        e.adjoint(component=3)
    assert all(torch.equal(x, y) for x, y in zip(before, e.state()))
    e.forward_record(T, ckpt, kap)
    g = e.adjoint(component=3)
    assert torch.isfinite(g).all()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_stored_window_gives_the_checkpointed_gradients(precision):
    """The same window differentiated from its stored trajectory and by
    checkpointed replay: FP64 gradients agree to rounding (only the order of
    the FP64 sums differs); FP32 ones to the path's tolerance, since a
    checkpointed reverse pass restarts the backward anchor advection from each
    segment's FP32 anchors."""
    N, M, T = 16, 48, 250
    kap = _shear(0.25)
    got = {}
    for ckpt in (50, T):
        e = _ens(N, M, precision=precision, seed=21, corr_levels=0, max_steps_per_launch=60).init()
        e.forward_record(T, ckpt, kap)
        got[ckpt] = e.adjoint(component=3).cpu().numpy()
    _check(got[T], got[50], 1e-12 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("ckpt", [7, 30], ids=["checkpointed", "stored"])
def test_adjoint_edge_cases_fp64(ckpt):
    """N = 2 chains (both beads are ends), a ragged launch (five N = 128
    chains: the second group holds one; seven N = 8 chains: a wave partly
    filled), a window that starts at an odd step after 3 plain steps (so no
    initial-anchor term), and a last segment shorter than the others
    (30 = 4 x 7 + 2)."""
    lengths = [2] * 3 + [128] * 5 + [8] * 7
    kap = _shear(0.2)
    e = _ens(np.array(lengths), precision="fp64", seed=27, corr_levels=0).init()
    e.step(3, kap)
    e.forward_record(30, ckpt, kap)
    got = e.adjoint(component=3).cpu().numpy()
    o = oracle.Ensemble(lengths, seed=27).init()
    for _ in range(3):
        o.step(kap)
    Rt, At, St = o.run_record(30, kap)
    gk, gns = o.adjoint(Rt, At, St, kap, step0=3, comp=3, init_window=False)
    want = np.concatenate([gk.reshape(len(lengths), 9), gns[:, None]], axis=1)
    assert np.array_equal(e.state()[2].cpu().numpy(), o.S)
    _check(got, want, 1e-9)


@pytest.mark.parametrize("ckpt", [1, 4], ids=["checkpointed", "stored"])
def test_one_step_window_fp64(ckpt):
    """The shortest window: one step, as one checkpoint segment or stored."""
    N, M = 10, 16
    kap = _shear(0.5)
    e = _ens(N, M, precision="fp64", seed=29, corr_levels=0).init()
    e.forward_record(1, ckpt, kap)
    got = e.adjoint(component=3).cpu().numpy()
    want, _ = _oracle_grad([N] * M, 29, 1, kap, 3)
    _check(got, want, 1e-9)


@pytest.mark.parametrize("ckpt", [40, 200], ids=["checkpointed", "stored"])
def test_reverse_pass_leaves_the_recording_intact(ckpt):
    """The replay reads each checkpoint in place and writes only the
    trajectory, so a second reverse pass over the same recording (here after
    one for another component) gives bitwise the same gradients, and the
    ensemble's own state is untouched."""
    N, M, T = 12, 32, 200
    kap = _shear(0.2)
    e = _ens(N, M, precision="fp32", seed=17, corr_levels=0).init()
    e.forward_record(T, ckpt, kap)
    state = [x.clone() for x in e.state()]
    g1 = e.adjoint(component=3).cpu().numpy()
    e.adjoint(component=0)
    g2 = e.adjoint(component=3).cpu().numpy()
    assert np.array_equal(g1, g2)
    assert all(torch.equal(x, y) for x, y in zip(state, e.state()))


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_stored_window_survives_a_mapping_change(precision, rtol):
    """A stored window's destruction log is in slot order, which every mapping
    shares: recorded at 32 lanes x 1 bead and differentiated at 16 x 2, it
    gives the gradients of the unchanged mapping (up to the order of the FP64
    sums).  The window holds steps in which one chain loses several springs,
    where the order matters."""
    N, M, T = 24, 64, 400
    kap = _shear(0.3)
    got = []
    for remap in (False, True):
        e = _ens(N, M, precision=precision, seed=13, corr_levels=0).init()
        e.set_mapping(2, 32, 32, 1)
        e.forward_record(T, T, kap)
        if remap:
            off = e._rec_p - e._rec_t.data_ptr()
            rows = e._rec_t[off:off + (T + 1) * N * M].view(T + 1, M, N).cpu().numpy().astype(np.int8)
            gone = (rows[:-1] >= 0) & (rows[1:] < 0)
            assert (gone.sum(axis=2) >= 2).any()
            e.set_mapping(2, 32, 16, 2)
        got.append(e.adjoint(component=3).cpu().numpy())
    _check(got[1], got[0], rtol)


@pytest.mark.parametrize("ckpt", [48, 200], ids=["checkpointed", "stored"])
@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_adjoint_under_the_k1_construction_rule(precision, rtol, ckpt):
    """The reverse pass replays recorded slot states, whatever rule decided
    them: a window recorded under the K = 1 rule differentiates like the
    oracle's run under the same rule, replayed or stored."""
    N, M, T = 10, 24, 200  # segments 48, 48, 48, 48, 8, or one stored window
    kap = _shear(0.2)
    e = _ens(N, M, precision=precision, seed=8, corr_levels=0, construct_rule=1).init()
    e.forward_record(T, ckpt, kap)
    got = e.adjoint(component=3).cpu().numpy()
    o = oracle.Ensemble([N] * M, seed=8, construct_rule=1).init()
    Rt, At, St = o.run_record(T, kap)
    gk, gns = o.adjoint(Rt, At, St, kap, comp=3)
    want = np.concatenate([gk.reshape(M, 9), gns[:, None]], axis=1)
    assert np.array_equal(e.state()[2].cpu().numpy(), o.S)  # same events
    _check(got, want, rtol)


def test_free_running_finite_differences_match_the_adjoint_where_no_decision_flips():
    """Central differences of the free-running forward (rate +- h, N_s +- h, the
    same random streams) per chain equal the pathwise adjoint on every chain
    whose slot row never differed from the unperturbed run's; chains where a
    decision flipped carry the jump the pathwise gradient omits (reading R18).
    FP64, 512 chains x N = 16, 300 steps under shear 0.3, h = 1e-6: the
    differences' truncation error is O(h^2) and their rounding error about
    1e-16 |J| / h, so the bar is 1e-6 of the gradients' rms."""
    M, N, T, g0, ns, h = 512, 16, 300, 0.3, 0.5, 1e-6

    def kap(g):
        k = torch.zeros(1, 9, dtype=torch.float64, device="cuda")
        k[0, 1] = g
        return k

    rec = _ens(N, M, precision="fp64", seed=31, corr_levels=0, ns=ns).init()
    rec.forward_record(T, 50, kap(g0))
    grad = rec.adjoint(component=3).cpu().numpy()
    rec.close()
    params = {"base": (g0, ns), "g-": (g0 - h, ns), "g+": (g0 + h, ns), "n-": (g0, ns - h), "n+": (g0, ns + h)}
    runs = {k: _ens(N, M, precision="fp64", seed=31, corr_levels=0, ns=v[1]).init() for k, v in params.items()}
    flipped = {k: torch.zeros(M, dtype=torch.bool, device="cuda") for k in params if k != "base"}
    for _ in range(T):
        for k, e in runs.items():
            e.step(1, kap(params[k][0]))
        S0 = runs["base"].state()[2].view(M, N)
        for k in flipped:
            flipped[k] |= (runs[k].state()[2].view(M, N) != S0).any(dim=1)
    J = {k: e.stress()[:, 3].cpu().numpy() for k, e in runs.items()}
    for col, lo, hi in ((1, "g-", "g+"), (9, "n-", "n+")):
        kept = ~(flipped[lo] | flipped[hi]).cpu().numpy()
        assert kept.sum() >= M // 2, kept.sum()
        fd = (J[hi] - J[lo]) / (2 * h)
        rms = np.sqrt(np.mean(grad[:, col] ** 2))
        err = np.abs(fd[kept] - grad[kept, col]).max() / rms
        assert err <= 1e-6, (col, err, int(kept.sum()))
