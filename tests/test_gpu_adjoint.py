"""GPU pathwise adjoint (recorded window, checkpointed replay, reverse pass)
against the oracle's discrete adjoint on the same seeded inputs.

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


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_adjoint_matches_oracle_shear(precision, rtol):
    N, M, T, ckpt = 12, 24, 300, 64  # segments 64, 64, 64, 64, 44
    kap = _shear(0.3)
    e = _ens(N, M, precision=precision, seed=5, corr_levels=0).init()
    e.forward_record(T, ckpt, kap)
    got = e.adjoint(component=3).cpu().numpy()
    want, o = _oracle_grad([N] * M, 5, T, kap, 3)
    S_end = e.state()[2].cpu().numpy()
    assert np.array_equal(S_end, o.S)  # same events
    _check(got, want, rtol)


def test_adjoint_matches_oracle_mixed_lengths_elongation_fp64():
    N = [5, 16, 33, 70, 128, 9, 40, 100] * 3
    kap = np.diag([0.02, -0.01, -0.01])
    e = _ens(N, precision="fp64", seed=9, corr_levels=0).init()
    e.forward_record(150, 50, kap)
    got = e.adjoint(component=0).cpu().numpy()
    want, _ = _oracle_grad(N, 9, 150, kap, 0)
    _check(got, want, 1e-9)


def test_forward_record_advances_exactly_like_step():
    kap = _shear(0.2)
    a = _ens(20, 32, precision="fp32", seed=3, corr_levels=4, corr_batches=4, sample_every=5).init()
    b = _ens(20, 32, precision="fp32", seed=3, corr_levels=4, corr_batches=4, sample_every=5).init()
    a.forward_record(230, 40, kap)
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


def test_adjoint_rejects_a_changed_recording_and_keeps_the_ensemble():
    """A slot row changed after ssp_forward_record (an impossible state, 100 in
    a chain of N = 8) is caught where the replay and the adjoint read it (both
    kernels check a row before using it, and read a bad entry as an empty
    slot): ssp_adjoint fails, the ensemble's own state is untouched, and a new
    recording differentiates normally."""
    from paper_1106_2899_amd._lib import SspError

    N, M, T, ckpt = 8, 64, 40, 10
    kap = _shear(0.1)
    e = _ens(N, M, precision="fp32", seed=31, corr_levels=0).init()
    e.forward_record(T, ckpt, kap)
    before = [x.clone() for x in e.state()]
    # slot rows: the first region of the recording buffer, [T + 1][N * M] int8
    off = e._rec_p - e._rec_t.data_ptr()
    rows = e._rec_t[off:off + (T + 1) * N * M].view(T + 1, N * M)
    rows[20, 3] = 100
    torch.cuda.synchronize()
    with pytest.raises(SspError, match="recorded slot rows"):
        e.adjoint(component=3)
    assert all(torch.equal(x, y) for x, y in zip(before, e.state()))
    e.forward_record(T, ckpt, kap)
    g = e.adjoint(component=3)
    assert torch.isfinite(g).all()


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_adjoint_under_the_k1_construction_rule(precision, rtol):
    """The reverse pass replays recorded slot states, whatever rule decided
    them: a window recorded under the K = 1 rule differentiates like the
    oracle's run under the same rule."""
    N, M, T, ckpt = 10, 24, 200, 48  # segments 48, 48, 48, 48, 8
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
