"""Start-up shear, steady viscosity, <Z> under flow and the Cox-Merz check
(Sec. 4.1) run through the library."""
import math

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_startup_shear_matches_oracle_fp64():
    """eta(t, gdot) = <sigma_xy(t)>/gdot and the final <Z> of the driver equal
    the oracle's on the same seeded run."""
    _need_gpu()
    from paper_1106_2899_amd.rheology import startup_shear
    N, M, rate, steps, every = 16, 64, 0.05, 2000, 10
    got = startup_shear(N, M, rate, steps, sample_every=every, precision="fp64", seed=7)
    o = oracle.Ensemble([N] * M, seed=7).init()
    z_eq = (o.S >= 0).sum() / M
    kap = np.zeros((3, 3))
    kap[0, 1] = rate
    s = o.run(steps, kappa=kap, sample_every=every)
    want = s[:, :, 3].mean(axis=1) / rate
    np.testing.assert_allclose(got.eta_plus, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
    assert got.z_eq == pytest.approx(z_eq, abs=0) and got.z_mean == pytest.approx((o.S >= 0).sum() / M, abs=0)
    np.testing.assert_allclose(got.t, (np.arange(steps // every) + 1) * every * 0.01)


def test_springs_under_shear_against_the_paper():
    """Against the numbers the paper prints for N = 80 (its CPU runs, K = 1
    construction): <Z>_eq = 20 and steady <Z> = 8.7, 4.2, 1.6 at
    gdot = 0.01, 0.1, 1 (no error bars given).  The runs go well past the
    transient (strains 600, 40 and 6), which at gdot = 1 lasts a few 1e5 steps:
    the stretched chain holds its springs until they slide off the ends."""
    _need_gpu()
    from paper_1106_2899_amd.rheology import startup_shear
    for rate, steps, z_paper in [(1.0, 600000, 1.6), (0.1, 400000, 4.2), (0.01, 600000, 8.7)]:
        r = startup_shear(80, 1024, rate, steps, sample_every=100, seed=11, construct_rule=1)
        print(f"N=80 gdot={rate}: <Z> = {r.z_mean:.2f} (paper {z_paper}), eq {r.z_eq:.2f}, eta = {r.eta:.2f} +- {r.eta_err:.2f}")
        assert r.z_eq == pytest.approx(20.0, rel=0.05)
        assert r.z_mean == pytest.approx(z_paper, rel=0.15)


def test_cox_merz_holds_at_low_rate():
    """In the linear regime the steady viscosity equals the zero-shear
    viscosity from the Green-Kubo modulus (Sec. 4.1: Cox-Merz holds for small
    rates; both tend to eta_0 = int G dt)."""
    _need_gpu()
    from paper_1106_2899_amd.ensemble import Ensemble
    from paper_1106_2899_amd.rheology import cox_merz, startup_shear
    N, M = 16, 16384
    e = Ensemble(N, M, precision="fp32", seed=5, sample_every=10, corr_levels=16, corr_batches=16)
    e.init()
    e.step(200000)
    lve = e.linear_viscoelasticity([0.002], 50.0, 150.0)
    e.close()
    r = startup_shear(N, M, 0.002, 200000, sample_every=10, seed=6)
    cm = cox_merz([r], lve["eta_abs"])
    print("N=16: eta_0", lve["eta0"], "|eta*(0.002)|", lve["eta_abs"][0], "eta(0.002)", r.eta, "+-", r.eta_err,
          "tau_d", lve["tau_d"])
    assert r.eta == pytest.approx(lve["eta0"], abs=4.0 * r.eta_err + 0.1 * lve["eta0"])
    assert cm["ratio"][0] == pytest.approx(1.0, abs=4.0 * r.eta_err / r.eta + 0.1)
