"""GPU observables and launch configurations against the FP64 oracle.

Covers: the multiple-tau correlator (G(t) in the Green-Kubo form with the
virtual stress), per-element stress series (viscosity growth), the stress
read-out, every chain-to-wavefront mapping (W = 8, 16, 32, 64 lanes per
chain; two beads per lane for N > 64) with mixed shear/elongation elements,
bitwise invariance to graph replay and launch chunking, and the non-finite
latch.  The oracle runs the same seeded inputs on its own.
"""
import numpy as np
import pytest

import oracle

from _corr import oracle_G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ens(N, M=None, **kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1106_2899_amd.ensemble import Ensemble
    return Ensemble(N, M, **kw)


def _oracle_G(samples, levels, virtual=False):
    """G[l][k] = sum over chains and xy, yz, zx of C / (3 M cnt), C the
    multiple-tau correlation of x = sigma (virtual: x = sigma^v) with
    y = sigma + sigma^v."""
    T, M, _ = samples.shape
    tot = np.zeros((levels, 16))
    cnt = None
    for k in range(M):
        for c in range(3):
            x = samples[:, k, (9 if virtual else 3) + c]
            y = samples[:, k, 3 + c] + samples[:, k, 9 + c]
            C, n = oracle.multitau(x, y, levels=levels, lags=16)
            tot += C
            cnt = n
    with np.errstate(invalid="ignore", divide="ignore"):
        G = np.where(cnt > 0, tot / (3.0 * M * np.maximum(cnt, 1)), 0.0)
    return G, cnt


def test_chunking_and_graph_invariance_bitwise():
    kw = dict(precision="fp32", seed=4, sample_every=3, corr_levels=6, corr_batches=4)
    kap = [[0, 0.2, 0], [0, 0, 0], [0, 0, 0]]
    a = _ens(20, 64, use_graph=True, **kw).init()
    b = _ens(20, 64, use_graph=False, max_steps_per_launch=7, **kw).init()
    a.step(300, kap)
    for _ in range(6):
        b.step(50, kap)
    for x, y in zip(a.state(), b.state()):
        assert torch.equal(x, y)
    ca, cb = a.correlator(), b.correlator()
    assert np.array_equal(ca["G"], cb["G"]) and np.array_equal(ca["counts"], cb["counts"])
    # replaying the cached graph continues the same trajectory
    a.step(300, kap)
    for _ in range(6):
        b.step(50, kap)
    for x, y in zip(a.state(), b.state()):
        assert torch.equal(x, y)


@pytest.mark.parametrize("steps", [1, 7, 300, 2000])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_persistent_schedule_equals_plain_launches_bitwise(precision, steps):
    """ssp_step under the persistent schedule (units of wavefronts' chains
    taken from a queue) and under one wavefront per chain group give the same
    state, correlator and element series bit for bit: mixed lengths (several
    mapping groups), mixed flows, sampling every 3 steps, launches from one
    step to 2000.  With fewer wave tasks than wavefront slots every launch is
    one time chunk; time chunks are covered by the test below."""
    N = [8, 16, 24, 32, 64, 100] * 40
    M = len(N)
    offs = np.array([0, M // 3, 2 * M // 3, M])
    kap = np.zeros((3, 9))
    kap[0, 1] = 0.4
    kap[1, [0, 4, 8]] = [0.02, -0.01, -0.01]
    kw = dict(precision=precision, seed=29, sample_every=3, corr_levels=8, corr_batches=4, series_capacity=1000,
              n_elements=3, element_offsets=offs, max_steps_per_launch=max(1, steps))
    a = _ens(N, **kw).init()
    b = _ens(N, **kw).init()
    b.set_schedule(False)
    for e in (a, b):
        e.step(steps, kap)
        e.step(steps)
    for x, y in zip(a.state(), b.state()):
        assert torch.equal(x, y)
    assert np.array_equal(a.correlator()["G"], b.correlator()["G"])
    assert torch.equal(a.element_series(), b.element_series())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_persistent_schedule_time_chunks_equal_plain_launches_bitwise(precision):
    """More wave tasks (7000) than wavefront slots, so that the persistent
    schedule splits each 2000-step launch into time chunks whose units wait
    for their chains' previous chunk: the same state, correlator and element
    series as one wavefront per chain group, bit for bit."""
    N = [32] * 14000
    M = len(N)
    offs = np.array([0, M // 2, M])
    kap = np.zeros((2, 9))
    kap[0, 1] = 0.3
    kw = dict(precision=precision, seed=31, sample_every=10, corr_levels=8, corr_batches=4, series_capacity=500,
              n_elements=2, element_offsets=offs, max_steps_per_launch=2000)
    a = _ens(N, **kw).init()
    b = _ens(N, **kw).init()
    b.set_schedule(False)
    for e in (a, b):
        e.step(2000, kap)
        e.step(2000)
    for x, y in zip(a.state(), b.state()):
        assert torch.equal(x, y)
    assert np.array_equal(a.correlator()["G"], b.correlator()["G"])
    assert torch.equal(a.element_series(), b.element_series())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_run_at_rest_equals_a_zero_velocity_gradient_table_bitwise(precision):
    """ssp_step with no table (the variant compiled without the flow terms)
    and with an all-zero table (the flow variant, whose flow branch is then
    skipped) give the same trajectory and correlator bit for bit."""
    kw = dict(precision=precision, seed=19, sample_every=2, corr_levels=6, corr_batches=4)
    a = _ens(24, 40, **kw).init()
    b = _ens(24, 40, **kw).init()
    a.step(400)
    b.step(400, np.zeros(9))
    for x, y in zip(a.state(), b.state()):
        assert torch.equal(x, y)
    assert np.array_equal(a.correlator()["G"], b.correlator()["G"])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_flowing_and_resting_chains_in_one_wavefront(precision):
    """Chains at rest that share wavefronts with sheared chains (8 lanes per
    chain: eight chains per wavefront, elements of three chains) follow the
    same trajectory as in an ensemble at rest."""
    N, M = 8, 48
    offs = np.arange(0, M + 1, 3)
    E = len(offs) - 1
    kap = np.zeros((E, 9))
    kap[::2, 1] = 0.7  # every other element sheared
    kw = dict(precision=precision, seed=23, corr_levels=0)
    a = _ens(N, M, n_elements=E, element_offsets=offs, **kw).init()
    b = _ens(N, M, **kw).init()
    a.step(300, kap)
    b.step(300)
    Ra, Aa, Sa = (x.cpu().numpy() for x in a.state())
    Rb, Ab, Sb = (x.cpu().numpy() for x in b.state())
    rest = np.repeat(np.arange(E) % 2 == 1, 3 * N)
    assert np.array_equal(Sa[rest], Sb[rest])
    assert np.array_equal(Ra[rest], Rb[rest])
    occ = rest & (Sa >= 0)
    assert np.array_equal(Aa[occ], Ab[occ])


@pytest.mark.parametrize("M,batches", [(32, 4), (100, 7)])
def test_correlator_and_batch_means_error_match_oracle_fp64(M, batches):
    """G(t) and its batch-means error G_err (standard error of the means of
    `batches` contiguous equal chain groups; 100 chains in 7 groups makes the
    groups unequal) against the same definitions applied to the oracle's
    samples of the same chains."""
    N, every, steps, L = 8, 3, 3000, 10
    e = _ens(N, M, precision="fp64", seed=6, sample_every=every, corr_levels=L, corr_batches=batches).init()
    e.step(steps)
    got = e.correlator()
    o = oracle.Ensemble([N] * M, seed=6).init()
    s = o.run(steps, sample_every=every)
    G, G_err, cnt = oracle_G(s, L, batches=batches)
    assert np.array_equal(got["counts"], cnt)
    np.testing.assert_allclose(got["G"], G, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(got["tau"][0], np.arange(16) * every * 0.01)
    ok = cnt > 1
    assert np.all(G_err[ok] > 0)
    np.testing.assert_allclose(got["G_err"], G_err, rtol=1e-8, atol=1e-12)


def test_virtual_stress_channel_matches_oracle_fp64():
    """The corr_virtual channel <sigma^v(t) [sigma + sigma^v](0)> and the
    relative virtual-stress contribution Gv / G (Sec. 4.1) against the
    oracle's multiple-tau correlation of the same samples; turning the channel
    on leaves G(t) unchanged."""
    M, N, every, steps, L = 32, 8, 3, 3000, 10
    e = _ens(N, M, precision="fp64", seed=6, sample_every=every, corr_levels=L, corr_batches=4,
             corr_virtual=True).init()
    e.step(steps)
    got = e.correlator_virtual()
    o = oracle.Ensemble([N] * M, seed=6).init()
    s = o.run(steps, sample_every=every)
    Gv, cnt = _oracle_G(s, L, virtual=True)
    G, _ = _oracle_G(s, L)
    np.testing.assert_allclose(got["Gv"], Gv, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(e.correlator()["G"], G, rtol=1e-9, atol=1e-11)
    ok = (cnt > 0) & (np.abs(G) > 1e-3)
    np.testing.assert_allclose(got["dG_v"][ok], Gv[ok] / G[ok], rtol=1e-8)
    assert np.all(np.isnan(got["dG_v"][cnt == 0]))  # lags without data
    assert np.all(got["Gv_err"][cnt > 0] >= 0)
    plain = _ens(N, M, precision="fp64", seed=6, sample_every=every, corr_levels=L, corr_batches=4).init()
    with pytest.raises(Exception):
        plain.correlator_virtual()


def test_correlator_matches_oracle_fp32_statistically_close():
    M, N, every, steps, L = 64, 16, 2, 2000, 8
    e = _ens(N, M, precision="fp32", seed=8, sample_every=every, corr_levels=L, corr_batches=8).init()
    e.step(steps)
    got = e.correlator()
    o = oracle.Ensemble([N] * M, seed=8).init()
    G, cnt = _oracle_G(o.run(steps, sample_every=every), L)
    # same trajectories up to FP32 rounding (1e-5 relative per step) and rare ties
    ok = cnt > 0
    np.testing.assert_allclose(got["G"][ok], G[ok], rtol=1e-3, atol=1e-3 * np.abs(G[ok]).max())


def test_element_series_matches_oracle_fp64():
    E, per, N, steps, every = 4, 16, 12, 500, 5
    rates = [0.0, 0.05, 0.5, 2.0]
    kap = np.zeros((E, 3, 3))
    kap[:, 0, 1] = rates
    e = _ens(N, E * per, n_elements=E, precision="fp64", seed=10, sample_every=every, corr_levels=0,
             series_capacity=200).init()
    e.step(steps, kap)
    ser = e.element_series().cpu().numpy()
    assert ser.shape == (E, steps // every, 6)
    o = oracle.Ensemble([N] * (E * per), seed=10).init()
    s = o.run(steps, kappa=np.repeat(kap.reshape(E, 9), per, axis=0), sample_every=every)
    want = s[:, :, :6].reshape(steps // every, E, per, 6).sum(axis=2).transpose(1, 0, 2)
    np.testing.assert_allclose(ser, want, rtol=1e-10, atol=1e-9)


def test_stress_readout_matches_oracle_fp64():
    M, N = 40, 24
    e = _ens(N, M, precision="fp64", seed=12, corr_levels=0).init()
    e.step(200)
    o = oracle.Ensemble([N] * M, seed=12).init()
    o.run(200, keep_samples=False)
    np.testing.assert_allclose(e.stress().cpu().numpy(), o.stress(), rtol=1e-11, atol=1e-10)


LENGTHS = [2, 5, 8, 9, 15, 16, 17, 24, 32, 33, 48, 64, 65, 90, 127, 128]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_mapping_mixed_flows(precision):
    N = LENGTHS * 4
    M = len(N)
    offs = [0, M // 2, M]
    kap = np.stack([np.array([[0, 0.3, 0], [0, 0, 0], [0, 0, 0]]), np.diag([0.05, -0.025, -0.025])])
    e = _ens(N, n_elements=2, element_offsets=offs, precision=precision, seed=14, corr_levels=0).init()
    o = oracle.Ensemble(N, seed=14).init()
    kchain = np.repeat(kap.reshape(2, 9), [M // 2, M - M // 2], axis=0)
    steps = 300
    e.step(steps, kap)
    o.run(steps, kappa=kchain, keep_samples=False)
    R, A, S = (x.cpu().numpy() for x in e.state())
    from paper_1106_2899_amd.ensemble import _invariants
    bg, dg, Sg = _invariants(R, A, S, np.array(N), e.offsets)
    bo, do, So = _invariants(o.R, o.A, o.S, np.array(N), o.off)
    tol = 1e-12 if precision == "fp64" else 1e-5
    same_chain = np.array([np.array_equal(Sg[e.offsets[k]:e.offsets[k] + N[k]], So[o.off[k]:o.off[k] + N[k]])
                           for k in range(M)])
    if precision == "fp64":
        assert same_chain.all()
    else:
        assert same_chain.sum() >= M - 3
    for k in np.nonzero(same_chain)[0]:
        sl = slice(e.offsets[k], e.offsets[k] + N[k])
        b_ok = ~np.isnan(bo[sl][:, 0])
        err = np.abs(bg[sl][b_ok] - bo[sl][b_ok]) / np.maximum(np.abs(bo[sl][b_ok]), 0.58)
        assert err.max() <= tol, (k, N[k], err.max())
        occ = So[sl] >= 0
        if occ.any():
            err = np.abs(dg[sl][occ] - do[sl][occ]) / np.maximum(np.abs(do[sl][occ]), 0.58)
            assert err.max() <= tol, (k, N[k], err.max())


def test_nonfinite_state_is_reported():
    from paper_1106_2899_amd import SspError
    e = _ens(16, 8, precision="fp32", seed=1, corr_levels=0).init()
    e.step(2000, np.diag([400.0, -200.0, -200.0]))  # elongation far beyond the Rouse stability limit
    with pytest.raises(SspError) as ei:
        e.stress()
    assert ei.value.code == -4


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_trajectory_does_not_depend_on_the_mapping(precision):
    """Every mapping that holds these chains, in both precisions (each kernel
    variant with its own register budget and spills): the state is bitwise
    the same; the element series (stress sampled every 5 steps) agrees to
    1e-12, since a mapping may change the order of the FP64 lane sums."""
    N = [20, 24, 31, 17] * 16
    kap = [[0, 0.4, 0], [0, 0, 0], [0, 0, 0]]
    ref = ref_ser = None
    for W, B in [(32, 1), (64, 1), (16, 2), (32, 2), (64, 2)]:
        e = _ens(N, precision=precision, seed=21, corr_levels=0, sample_every=5, series_capacity=30)
        e.set_mapping(17, 31, W, B)
        e.init().step(150, kap)
        st = [x.cpu() for x in e.state()]
        ser = e.element_series().cpu().numpy()
        if ref is None:
            ref, ref_ser = st, ser
        else:
            for x, y in zip(ref, st):
                assert torch.equal(x, y), (W, B)
            np.testing.assert_allclose(ser, ref_ser, rtol=1e-12, atol=1e-12 * np.abs(ref_ser).max())
        e.close()


def test_autotuner_picks_a_valid_mapping_and_keeps_results():
    from paper_1106_2899_amd import autotune
    N = np.array([12, 30, 50, 100] * 64, dtype=np.int32)
    e = _ens(N, precision="fp32", seed=22, corr_levels=0)
    res = autotune.tune(e, steps=50, probe_chains=256)
    for (lo, hi), (W, B) in res.choices.items():
        assert W * B >= N[(N >= lo) & (N <= hi)].max()
    e.init().step(100)
    f = _ens(N, precision="fp32", seed=22, corr_levels=0).init().step(100)
    for x, y in zip(e.state(), f.state()):
        assert torch.equal(x, y)
