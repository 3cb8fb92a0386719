"""Pins of the linear-viscoelasticity oracle (Sec. 4.1 relations for G', G'',
eta_0 and tau_d), independent of the HIP path."""
import math

import numpy as np
import pytest

import oracle
from oracle import moduli as M

SAMPLE_DT = 0.1  # n_s = 10 steps of dt = 0.01


def _maxwell(t, g, tau):
    return g * np.exp(-t / tau)


def test_grid_is_the_lags_with_data():
    """Level 0 lags 0..15 and level l >= 1 lags 8..15, exactly the lags of the
    multiple-tau correlator that hold at least one product."""
    samples, levels = 1000, 12
    t, idx = M.multitau_grid(levels, samples, SAMPLE_DT)
    _, cnt = oracle.multitau(np.ones(samples), np.ones(samples), levels=levels, lags=16)
    want = [l * 16 + k for l in range(levels) for k in range(0 if l == 0 else 8, 16) if cnt[l, k] > 0]
    assert list(idx) == want
    assert np.all(np.diff(t) > 0)
    np.testing.assert_allclose(t, [(i % 16) * 2 ** (i // 16) * SAMPLE_DT for i in idx], rtol=1e-15)


def test_series_for_sin_minus_hcos():
    # against the difference in extended precision where that keeps >= 14 digits
    for h in [0.01, 0.1, 0.3, 0.49, 0.499999, 0.5, 0.51, 1.0, 3.0]:
        x = np.longdouble(h)
        want = float(np.sin(x) - x * np.cos(x))
        assert M._s3(h) == pytest.approx(want, rel=1e-13, abs=0.0)
    # small h: sin h - h cos h = (h^3/3)(1 - h^2/10 + O(h^4))
    for h in [1e-8, 1e-6, 1e-4, 1e-3]:
        assert abs(M._s3(h) / (h**3 / 3.0) - 1.0 + h * h / 10.0) < h**4 + 1e-15


def test_matches_plain_trapezoid_on_a_fine_uniform_grid():
    """On a fine uniform grid the paper's literal rule (trapezoid of G sin and
    G cos) and the piecewise-linear-G integral agree to O(dt^2): their
    difference is the trapezoid error of G_lin sin(w t), whose second
    derivative carries 2 w G' cos(w t)."""
    t = np.arange(0.0, 400.0, 0.01)
    G = _maxwell(t, 1.5, 20.0) + _maxwell(t, 0.5, 2.0)
    for w in [0.01, 0.1, 0.5]:
        got = M.dynamic_moduli(t, G, [w])[0]
        gp = w * np.trapezoid(G * np.sin(w * t), t)
        gpp = w * np.trapezoid(G * np.cos(w * t), t)
        tol = 0.1 * 0.01**2
        assert got[0] == pytest.approx(gp, rel=tol)
        assert got[1] == pytest.approx(gpp, rel=tol)
    assert M.zero_shear_viscosity(t, G) == pytest.approx(np.trapezoid(G, t), rel=1e-13)


@pytest.mark.parametrize("g,tau", [(2.0, 50.0), (1.0, 5.0)])
def test_maxwell_closed_forms_on_the_multiple_tau_grid(g, tau):
    """A Maxwell mode G = g e^{-t/tau}: G' = g x^2/(1+x^2), G'' = g x/(1+x^2)
    with x = w tau, eta_0 = g tau, tau_d = tau.  The multiple-tau grid of a
    1e5-step run sampled every 10 steps carries G to within the linear
    interpolation error of its log spacing."""
    t, _ = M.multitau_grid(16, 10000, SAMPLE_DT)
    G = _maxwell(t, g, tau)
    om = 10.0 ** np.linspace(-4, 0, 17)
    out = M.dynamic_moduli(t, G, om)
    x = om * tau
    gp, gpp = g * x**2 / (1 + x**2), g * x / (1 + x**2)
    np.testing.assert_allclose(out[:, 0], gp, rtol=1e-2)
    ok = x <= 10.0
    np.testing.assert_allclose(out[ok, 1], gpp[ok], rtol=1e-2)
    np.testing.assert_allclose(out[:, 2], np.hypot(out[:, 0], out[:, 1]) / om, rtol=1e-14)
    assert M.zero_shear_viscosity(t, G) == pytest.approx(g * tau, rel=2e-3)
    assert M.longest_relaxation_time(t, G, 4 * tau, 20 * tau) == pytest.approx(tau, rel=1e-9)


def test_longest_relaxation_time_of_two_modes_and_degenerate_windows():
    t, _ = M.multitau_grid(16, 10000, SAMPLE_DT)
    G = _maxwell(t, 1.0, 3.0) + _maxwell(t, 0.2, 60.0)
    assert M.longest_relaxation_time(t, G, 400.0, 800.0) == pytest.approx(60.0, rel=1e-6)
    assert math.isnan(M.longest_relaxation_time(t, G, 5000.0, 6000.0))  # no points
    assert math.isnan(M.longest_relaxation_time(t, np.ones_like(t), 1.0, 100.0))  # slope 0
