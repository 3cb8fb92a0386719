"""G'(w), G''(w), |eta*(w)|, eta_0 and tau_d computed on the device
(ssp_linear_viscoelasticity, Sec. 4.1 relations) against the oracle's plain
evaluation of the same definitions on the same grid and the same G."""
import math

import numpy as np
import pytest

from oracle import moduli as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SAMPLE_EVERY, DT = 10, 0.01


def _ens(N, M_=None, **kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1106_2899_amd.ensemble import Ensemble
    return Ensemble(N, M_, **kw)


@pytest.fixture(scope="module")
def run():
    """64 chains of N = 8 run for 1e5 steps, a sample every 10 steps: 1e4
    samples on a 16-level multiple-tau grid."""
    e = _ens(8, 64, precision="fp64", seed=21, sample_every=SAMPLE_EVERY, corr_levels=16, corr_batches=4)
    e.init()
    e.step(100000)
    c = e.correlator()
    samples = int(c["counts"][0, 0])
    assert samples == 10000
    t, idx = M.multitau_grid(16, samples, SAMPLE_EVERY * DT)
    yield e, c, t, idx
    e.close()


def _check(got, t, G, om, t_lo, t_hi):
    want = M.dynamic_moduli(t, G, om)
    scale = M.moduli_error_scale(t, G, om)
    for q in range(2):  # rounding bound of the segment sums
        assert np.all(np.abs(got["Gp" if q == 0 else "Gpp"] - want[:, q]) <= 1e-12 * scale[:, q] + 1e-300)
    np.testing.assert_allclose(got["eta_abs"], want[:, 2], rtol=1e-10)
    assert got["eta0"] == pytest.approx(M.zero_shear_viscosity(t, G), rel=1e-13)
    tau = M.longest_relaxation_time(t, G, t_lo, t_hi)
    if math.isnan(tau):
        assert math.isnan(got["tau_d"])
    else:
        assert got["tau_d"] == pytest.approx(tau, rel=1e-10)


def test_moduli_of_a_maxwell_mode_on_the_device_grid(run):
    e, _, t, idx = run
    g, tau = 2.0, 50.0
    full = np.zeros(16 * 16)
    lag_t = np.array([(i % 16) * 2 ** (i // 16) * SAMPLE_EVERY * DT for i in range(256)])
    full[:] = g * np.exp(-lag_t / tau)
    om = 10.0 ** np.linspace(-4, 1, 26)
    got = e.linear_viscoelasticity(om, 4 * tau, 20 * tau, G=torch.tensor(full, device="cuda"))
    _check(got, t, full[idx], om, 4 * tau, 20 * tau)
    # and the closed forms, as far as the grid carries them
    x = om * tau
    ok = x <= 10.0
    np.testing.assert_allclose(got["Gp"][om <= 1.0], (g * x**2 / (1 + x**2))[om <= 1.0], rtol=1e-2)
    np.testing.assert_allclose(got["Gpp"][ok], (g * x / (1 + x**2))[ok], rtol=1e-2)
    assert got["tau_d"] == pytest.approx(tau, rel=1e-9)


def test_moduli_of_the_measured_relaxation_modulus(run):
    e, c, t, idx = run
    G = c["G"].ravel()
    om = 10.0 ** np.linspace(-3, 1, 21)
    got = e.linear_viscoelasticity(om, 5.0, 30.0)
    _check(got, t, G[idx], om, 5.0, 30.0)
    # G' rises to the short-time modulus, G'' is positive, eta_0 > 0
    assert np.all(got["Gpp"][:15] > 0) and got["eta0"] > 0


def test_degenerate_windows_and_arguments(run):
    e, _, _, _ = run
    got = e.linear_viscoelasticity([], 1e6, 2e6)  # no frequencies, empty window
    assert math.isnan(got["tau_d"]) and got["eta0"] > 0
    from paper_1106_2899_amd._lib import SspError
    with pytest.raises(SspError):
        e.linear_viscoelasticity([0.1], 2.0, 1.0)
