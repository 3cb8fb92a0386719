"""Pins of the FP64 oracle to facts the paper and mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors and an independent library implementation (Philox),
distribution laws (Box-Muller, the equilibrium sampler of Sec. 3.1),
the free energy of Sec. 2.1 (forces by finite differences), the Glauber
detailed-balance identity (Sec. 2.2), closed forms of the Euler-discretised
Rouse chain (springs off), the exact stationary law of the N = 2 slot Markov
chain (Sec. 3.1 substep 3 with K = C - Z, Sec. 3.2), and the linear-response
prediction of Sec. 2.3 (step strain vs. the Green-Kubo correlation that
includes the virtual stress).
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
DT, N0, NS, ZS = 0.01, 4.0, 0.5, 0.1


# ---------------------------------------------------------------- RNG ------

def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answer_vectors():
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert list(oracle.philox(ctr, key)) == want


def test_philox_matches_rocrand_host_implementation():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    rng = np.random.default_rng(123)
    cases = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "rr")
        subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-o", exe,
                               os.path.join(HERE, "rocrand_philox_ref.cpp")], cwd=d)
        inp = "\n".join(" ".join(str(int(x)) for x in row) for row in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(cases, out):
        want = [int(x) for x in line.split()]
        got = list(oracle.philox(row[:4], row[4:6]))
        assert got == want


def test_u01_grid_and_range():
    assert oracle.u01(0) == 0.5 * 2.0**-23
    assert oracle.u01(0xFFFFFFFF) == 1.0 - 0.5 * 2.0**-23
    assert oracle.u01(1 << 9) == 1.5 * 2.0**-23
    # exactly representable in binary32: (2k+1) < 2^24
    for w in [0, 1 << 9, 12345 << 9, 0xFFFFFFFF]:
        u = oracle.u01(w)
        assert float(np.float32(u)) == u


def test_box_muller_normals_are_standard():
    g = np.array([oracle.normals3(7, oracle.P_NOISE, i % 64, i // 64, 3) for i in range(60000)])
    assert np.all(np.isfinite(g))
    for c in range(3):
        x = g[:, c]
        assert abs(x.mean()) < 4.0 / math.sqrt(len(x))
        assert abs(x.var() - 1.0) < 4.0 * math.sqrt(2.0 / len(x))
        assert stats.kstest(x, "norm").pvalue > 1e-3
    # the three components are uncorrelated
    cc = np.corrcoef(g.T)
    assert np.max(np.abs(cc - np.eye(3))) < 4.0 / math.sqrt(len(g))


def test_streams_are_distinct_by_purpose_chain_step():
    a = oracle.block(1, oracle.P_NOISE, 3, 5, 7)
    assert not np.array_equal(a, oracle.block(1, oracle.P_SLOT, 3, 5, 7))
    assert not np.array_equal(a, oracle.block(1, oracle.P_NOISE, 3, 6, 7))
    assert not np.array_equal(a, oracle.block(1, oracle.P_NOISE, 3, 5, 8))
    assert not np.array_equal(a, oracle.block(2, oracle.P_NOISE, 3, 5, 7))
    # step counter uses both 32-bit halves
    assert not np.array_equal(oracle.block(1, oracle.P_NOISE, 0, 0, 1), oracle.block(1, oracle.P_NOISE, 0, 0, 1 << 32))


def test_step_pair_streams_layout_and_independence():
    """Per-step streams in step pairs (2k, 2k+1): the bead noise of the two
    steps is six Box-Muller normals of blocks NOISE(k) and NOISE2(k); the slot
    words are NOISE2(k) words 2, 3 at the even step and SLOT(k) words 0, 1 at
    the odd step.  The normals of both steps are standard and uncorrelated,
    also between the members of the Box-Muller pair that the two steps share."""
    def bm(wa, wb):
        r = math.sqrt(-2.0 * math.log(oracle.u01(wa)))
        t = 2.0 * math.pi * oracle.u01(wb)
        return r * math.cos(t), r * math.sin(t)

    for (i, c, k) in [(0, 0, 0), (5, 9, 123), (31, 70000, (1 << 33) + 7)]:
        x = oracle.block(4, oracle.P_NOISE, i, c, k)
        y = oracle.block(4, oracle.P_NOISE2, i, c, k)
        z = oracle.block(4, oracle.P_SLOT, i, c, k)
        a0, a1 = bm(x[0], x[1])
        a2, a3 = bm(x[2], x[3])
        a4, a5 = bm(y[0], y[1])
        np.testing.assert_allclose(oracle.step_noise(4, i, c, 2 * k), [a0, a1, a2], rtol=0, atol=1e-15)
        np.testing.assert_allclose(oracle.step_noise(4, i, c, 2 * k + 1), [a3, a4, a5], rtol=0, atol=1e-15)
        assert list(oracle.slot_words(4, i, c, 2 * k)) == [y[2], y[3]]
        assert list(oracle.slot_words(4, i, c, 2 * k + 1)) == [z[0], z[1]]

    n = 20000
    ev = np.array([oracle.step_noise(9, i % 32, i // 32, 40) for i in range(n)])
    od = np.array([oracle.step_noise(9, i % 32, i // 32, 41) for i in range(n)])
    g = np.hstack([ev, od])
    for col in range(6):
        assert abs(g[:, col].mean()) < 4.0 / math.sqrt(n)
        assert abs(g[:, col].var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
        assert stats.kstest(g[:, col], "norm").pvalue > 1e-3
    assert np.max(np.abs(np.corrcoef(g.T) - np.eye(6))) < 4.0 / math.sqrt(n)
    # slot words of the two steps are uniform and uncorrelated with each other
    u = np.array([[oracle.u01(w) for w in list(oracle.slot_words(9, i % 32, i // 32, 40)) +
                   list(oracle.slot_words(9, i % 32, i // 32, 41))] for i in range(n)])
    for col in range(4):
        assert stats.kstest(u[:, col], "uniform").pvalue > 1e-3
    assert np.max(np.abs(np.corrcoef(u.T) - np.eye(4))) < 4.0 / math.sqrt(n)


# -------------------------------------------------------- initial state ----

def test_equilibrium_sampler_laws():
    """Sec. 3.1 sampling procedure; laws of Sec. 2.1 (ideal chain bonds,
    Poisson Z, uniform S, Gaussian anchors)."""
    M, N = 20000, 8
    e = oracle.Ensemble([N] * M, seed=11).init()
    R = e.R.reshape(M, N, 3)
    assert np.all(R[:, 0, :] == 0.0)
    b = (R[:, 1:] - R[:, :-1]).ravel()
    assert stats.kstest(b / math.sqrt(1.0 / 3.0), "norm").pvalue > 1e-3
    S = e.S.reshape(M, N)
    Z = (S >= 0).sum(axis=1)
    # occupied slots are exactly 0..Z-1
    for k in range(0, M, 997):
        assert np.all(S[k, :Z[k]] >= 0) and np.all(S[k, Z[k]:] == -1)
    lam = N / N0
    pmf = np.array([math.exp(-lam) * lam**z / math.factorial(z) for z in range(N + 1)])
    pmf /= pmf.sum()
    obs = np.bincount(Z, minlength=N + 1)
    exp = pmf * M
    keep = exp > 5
    chi2 = (((obs - exp) ** 2 / exp)[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3
    s = S[S >= 0]
    cnt = np.bincount(s, minlength=N)
    chi2 = ((cnt - len(s) / N) ** 2 / (len(s) / N)).sum()
    assert stats.chi2.sf(chi2, N - 1) > 1e-3
    d = e.anchor_offsets()
    d = d[~np.isnan(d[:, 0])].ravel()
    assert stats.kstest(d / math.sqrt(NS / 3.0), "norm").pvalue > 1e-3


# ------------------------------------------------------- forces / flow -----

def _free_energy(R, A, S, ns):
    f = 1.5 * np.sum((R[1:] - R[:-1]) ** 2)
    for j, s in enumerate(S):
        if s >= 0:
            f += 1.5 / ns * np.sum((R[s] - A[j]) ** 2)
    return f


def _set_state(e, R, A, S):
    e.R[:] = R
    e.A[:] = A
    e.S[:] = S


def test_force_is_minus_gradient_of_free_energy():
    """Substep 1 drift equals -dF/dR (Sec. 2.1 free energy, Sec. 3.1)."""
    rng = np.random.default_rng(5)
    N = 6
    e = oracle.Ensemble([N], seed=3, n0=1e30)  # no creation: p = 0
    R = rng.normal(size=(N, 3))
    A = rng.normal(size=(N, 3))
    S = np.array([2, 2, -1, 0, 5, 3], dtype=np.int32)  # two springs share bead 2
    _set_state(e, R, A, S)
    e.step_index = 17
    e.step()
    g = np.array([oracle.step_noise(3, i, 0, 17) for i in range(N)])
    drift = (e.R - R - math.sqrt(2 * DT) * g) / DT
    h = 1e-5
    grad = np.zeros_like(R)
    for i in range(N):
        for c in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[i, c] += h
            Rm[i, c] -= h
            grad[i, c] = (_free_energy(Rp, A, S, NS) - _free_energy(Rm, A, S, NS)) / (2 * h)
    np.testing.assert_allclose(drift, -grad, rtol=1e-7, atol=1e-7)


def test_flow_term_orientation_and_anchor_advection():
    """kappa.R with (kappa.R)_a = sum_b kappa_ab R_b; simple shear
    kappa_xy = gdot moves x by gdot*y (Sec. 2.2 and the shear flow of
    Sec. 4.1); anchors are advected affinely."""
    rng = np.random.default_rng(8)
    N = 4
    R = rng.normal(size=(N, 3))
    A = rng.normal(size=(N, 3))
    S = np.array([1, -1, 3, -1], dtype=np.int32)
    kap = np.zeros((3, 3))
    kap[0, 1] = 0.7
    out = {}
    for name, k in [("flow", kap), ("rest", np.zeros((3, 3)))]:
        e = oracle.Ensemble([N], seed=4, n0=1e30, zeta_s=1e30)  # no hops, no reconstruction
        _set_state(e, R, A, S)
        e.step(k)
        out[name] = (e.R.copy(), e.A.copy())
    np.testing.assert_allclose(out["flow"][0] - out["rest"][0], DT * R @ kap.T, rtol=1e-12, atol=1e-14)
    dA = out["flow"][1] - A
    np.testing.assert_allclose(dA[[0, 2]], DT * A[[0, 2]] @ kap.T, rtol=1e-12, atol=1e-14)


def test_hop_detailed_balance_glauber():
    """P(S->S+1) exp(-F(S)) = P(S+1->S) exp(-F(S+1)) for the unclipped
    Glauber probabilities (Sec. 2.2 rates; Sec. 3.1 substep 2)."""
    rng = np.random.default_rng(9)
    N = 7
    for trial in range(20):
        R = rng.normal(size=(N, 3)) * 0.8
        a = rng.normal(size=3) * 0.5
        for s in range(N - 1):
            pu = oracle.hop_prob(R, a, s, +1, DT, NS, ZS)
            pd = oracle.hop_prob(R, a, s + 1, -1, DT, NS, ZS)
            F0 = 1.5 / NS * np.sum((R[s] - a) ** 2)
            F1 = 1.5 / NS * np.sum((R[s + 1] - a) ** 2)
            assert pu < 0.5 and pd < 0.5
            assert pu * math.exp(-F0) == pytest.approx(pd * math.exp(-F1), rel=1e-12)
        assert oracle.hop_prob(R, a, N - 1, +1, DT, NS, ZS) == 0.0
        assert oracle.hop_prob(R, a, 0, -1, DT, NS, ZS) == 0.0
    # zero energy difference: (dt/zeta_s)(1 - tanh 0) = dt/zeta_s
    R = np.zeros((3, 3))
    assert oracle.hop_prob(R, np.zeros(3), 1, +1, DT, NS, ZS) == pytest.approx(DT / ZS, rel=1e-15)
    # the 1/2 cap binds for large dt/zeta_s
    assert oracle.hop_prob(R, np.zeros(3), 1, +1, 0.4, NS, 0.1) == 0.5


# ------------------------------------------- discrete Rouse closed forms ---

def _rouse_modes(N, dt):
    p = np.arange(1, N)
    lam = 4.0 * np.sin(p * np.pi / (2 * N)) ** 2
    return lam, 1.0 - 3.0 * dt * lam


def rouse_corr(N, dt, n):
    """<sigma_xy(n dt) sigma_xy(0)> of the Euler-discretised Rouse chain in its
    stationary state: sum_p rho_p^(2n) / (1 - 1.5 dt lam_p)^2."""
    lam, rho = _rouse_modes(N, dt)
    return float(np.sum(rho ** (2 * n) / (1.0 - 1.5 * dt * lam) ** 2))


def rouse_normal(N, dt):
    lam, _ = _rouse_modes(N, dt)
    return float(np.sum(1.0 / (1.0 - 1.5 * dt * lam)) - N)


def _rouse_lyapunov(N, dt, lags):
    """The same stationary quantities by a different route: solve the discrete
    Lyapunov equation Sigma = M Sigma M^T + 2 dt B for the bond covariance of
    b' = M b + sqrt(2 dt) D w (B = D D^T, M = 1 - 3 dt B)."""
    import scipy.linalg as sl
    D = np.zeros((N - 1, N))
    for i in range(N - 1):
        D[i, i], D[i, i + 1] = -1.0, 1.0
    B = D @ D.T
    Mm = np.eye(N - 1) - 3.0 * dt * B
    Sig = sl.solve_discrete_lyapunov(Mm, 2.0 * dt * B)
    corr = [9.0 * float(np.sum((np.linalg.matrix_power(Mm, n) @ Sig) ** 2)) for n in lags]
    return 3.0 * float(np.trace(Sig)) - N, corr


def test_rouse_closed_forms_agree_with_lyapunov_solution():
    for N in (4, 8, 16):
        normal, corr = _rouse_lyapunov(N, DT, [0, 5, 100])
        assert rouse_normal(N, DT) == pytest.approx(normal, rel=1e-12)
        for n, c in zip([0, 5, 100], corr):
            assert rouse_corr(N, DT, n) == pytest.approx(c, rel=1e-10)


def _batch_se(per_chain, nb=32):
    b = np.array([x.mean() for x in np.array_split(per_chain, nb)])
    return b.mean(), b.std(ddof=1) / math.sqrt(nb)


@pytest.fixture(scope="module")
def rouse_run():
    N, M = 8, 1024
    e = oracle.Ensemble([N] * M, seed=21, n0=1e30).init()  # springs switched off
    e.run(600, keep_samples=False)                          # relax to the discrete stationary law
    s = e.run(4000, sample_every=5)                         # [800][M][12]
    return N, s


@pytest.mark.parametrize("lag_samples", [0, 1, 4, 10, 20])
def test_rouse_stress_autocorrelation_closed_form(rouse_run, lag_samples):
    N, s = rouse_run
    T = s.shape[0]
    off = s[:, :, 3:6]  # xy yz zx
    prod = (off[lag_samples:] * off[:T - lag_samples]).mean(axis=(0, 2))  # per chain
    est, se = _batch_se(prod)
    want = rouse_corr(N, DT, 5 * lag_samples)
    assert abs(est - want) < 4.0 * se + 1e-12, (est, want, se)
    if lag_samples == 0:
        # the discrete map differs from the continuous Rouse value N - 1
        assert abs(est - (N - 1)) > 4.0 * se


def test_rouse_mean_normal_stress_closed_form(rouse_run):
    N, s = rouse_run
    per_chain = s[:, :, 0:3].mean(axis=(0, 2))
    est, se = _batch_se(per_chain)
    want = rouse_normal(N, DT)
    assert want == pytest.approx(-0.7805449, abs=1e-6)
    assert abs(est - want) < 4.0 * se
    assert abs(est - (-1.0)) > 4.0 * se  # continuous equilibrium value -kBT


# ------------------------------------------ N = 2: exact slot Markov chain ---

def n2_stationary(dt=DT, n0=N0, zeta_s=ZS, rule=0):
    """Z of a 2-bead chain is an autonomous Markov chain (both beads are ends):
    each occupied slot is destroyed with min(dt/zeta_s, 1); springs created in
    the step are not destroyed in it.  Rule 0 (GPU rule, Sec. 3.2): each of the
    K = 2 - Z empty slots creates with probability 2 min(dt/(zeta_s n0 K), 1/2).
    Rule 1 (CPU rule, K = 1): one attempt while a slot is empty, creating with
    probability 2 min(dt/(zeta_s n0), 1/2)."""
    from math import comb
    cd = min(dt / zeta_s, 1.0)
    P = np.zeros((3, 3))
    for z in range(3):
        K = 2 - z if rule == 0 else (1 if z < 2 else 0)
        q = 2.0 * min(dt / (zeta_s * n0 * (K if rule == 0 else 1)), 0.5) if K > 0 else 0.0
        for d in range(z + 1):
            pd = comb(z, d) * cd**d * (1 - cd) ** (z - d)
            for c in range(K + 1):
                pc = comb(K, c) * q**c * (1 - q) ** (K - c)
                P[z, z - d + c] += pd * pc
    w, v = np.linalg.eig(P.T)
    pi = np.real(v[:, np.argmin(np.abs(w - 1))])
    return pi / pi.sum()


def test_n2_stationary_law_of_z():
    pi = n2_stationary()
    np.testing.assert_allclose(pi, [0.613472, 0.310881, 0.075648], atol=2e-6)
    M = 20000
    e = oracle.Ensemble([2] * M, seed=31).init()
    e.run(300, keep_samples=False)
    Zt = []
    for _ in range(60):
        e.run(25, keep_samples=False)
        Zt.append((e.S.reshape(M, 2) >= 0).sum(axis=1))
    Zt = np.array(Zt)  # [60][M]
    frac = np.stack([(Zt == z).mean(axis=0) for z in range(3)], axis=1)  # per chain
    for z in range(3):
        est, se = _batch_se(frac[:, z])
        assert abs(est - pi[z]) < 4.0 * se + 1e-4, (z, est, pi[z], se)


def test_n2_stationary_law_of_z_cpu_rule_and_detailed_balance_comparison():
    """The K = 1 construction rule (Sec. 3.2, CPU) as a variant: the oracle's
    N = 2 chains follow that rule's exact law, which differs from the GPU
    rule's; both approach the equilibrium law (Poisson(N/N0) truncated to
    0..2) linearly in dt, the K = 1 rule with about twice the bias."""
    pi1 = n2_stationary(rule=1)
    np.testing.assert_allclose(pi1, [0.611570, 0.314050, 0.074380], atol=2e-6)
    eq = np.array([1.0, 0.5, 0.125])
    eq /= eq.sum()
    bias = {}
    for dt in (0.01, 0.005, 0.0025):
        bias[dt] = [np.abs(n2_stationary(dt=dt, rule=r) - eq).max() for r in (0, 1)]
    for r in (0, 1):  # O(dt): halving dt halves the bias
        assert bias[0.005][r] / bias[0.01][r] == pytest.approx(0.5, abs=0.02)
        assert bias[0.0025][r] / bias[0.005][r] == pytest.approx(0.5, abs=0.02)
    assert bias[0.01][1] == pytest.approx(2.0 * bias[0.01][0], rel=0.05)

    M = 20000
    e = oracle.Ensemble([2] * M, seed=33, construct_rule=1).init()
    e.run(300, keep_samples=False)
    Zt = []
    for _ in range(60):
        e.run(25, keep_samples=False)
        Zt.append((e.S.reshape(M, 2) >= 0).sum(axis=1))
    Zt = np.array(Zt)
    frac = np.stack([(Zt == z).mean(axis=0) for z in range(3)], axis=1)
    pi0 = n2_stationary(rule=0)
    est1, se1 = _batch_se(frac[:, 1])
    for z in range(3):
        est, se = _batch_se(frac[:, z])
        assert abs(est - pi1[z]) < 4.0 * se + 1e-4, (z, est, pi1[z], se)
    # at most one spring is created per step
    e2 = oracle.Ensemble([8] * 2000, seed=34, construct_rule=1).init()
    for _ in range(50):
        before = e2.S.reshape(2000, 8) >= 0
        ev, _ = e2.step(want_events=True)
        created = (ev.reshape(2000, 8) & (oracle.EV_CREATE_FIRST | oracle.EV_CREATE_LAST)) > 0
        assert created.sum(axis=1).max() <= 1
        # ... and only by the lowest slot empty after the hops (hops keep the
        # occupancy, so that is the lowest slot empty at the start of the step)
        rows = np.nonzero(created.any(axis=1))[0]
        for r in rows:
            j = int(np.nonzero(created[r])[0][0])
            assert j == int(np.nonzero(~before[r])[0][0])
    assert abs(est1 - pi0[1]) > 3.0 * se1  # the two rules are distinguishable here


# ---------------------------------------- equilibrium with springs on ------

def _stationary_averages(N, M, dt, seed, t_eq=10.0, t_avg=20.0, every=0.25):
    """Time averages over [t_eq, t_eq + t_avg] (snapshots every `every` time
    units) of the per-chain observables, with standard errors over the
    independent chains: <Z>, the bond variance per component, the
    anchor-offset variance per component, and the share of springs on an end
    bead (the last two as ratio estimators)."""
    e = oracle.Ensemble([N] * M, dt=dt, seed=seed).init()
    e.run(int(round(t_eq / dt)), keep_samples=False)
    k, nsnap = int(round(every / dt)), int(round(t_avg / every))
    z, b2, d2, nd, ends, occn = (np.zeros(M) for _ in range(6))
    for _ in range(nsnap):
        e.run(k, keep_samples=False)
        S, R, A = e.S.reshape(M, N), e.R.reshape(M, N, 3), e.A.reshape(M, N, 3)
        occ = S >= 0
        z += occ.sum(axis=1)
        b2 += ((R[:, 1:] - R[:, :-1]) ** 2).mean(axis=(1, 2))
        RS = np.take_along_axis(R, np.where(occ, S, 0)[..., None], axis=1)
        d2 += (np.where(occ[..., None], RS - A, 0.0) ** 2).sum(axis=(1, 2))
        nd += 3 * occ.sum(axis=1)
        ends += (occ & ((S == 0) | (S == N - 1))).sum(axis=1)
        occn += occ.sum(axis=1)

    def mean_se(x):
        x = x / nsnap
        return x.mean(), x.std(ddof=1) / math.sqrt(M)

    def ratio_se(s, c):
        r = s.sum() / c.sum()
        return r, math.sqrt(((s - r * c) ** 2).sum() * M / (M - 1)) / c.sum()

    return {"Z": mean_se(z), "bond_var": mean_se(b2), "offset_var": ratio_se(d2, nd), "end_share": ratio_se(ends, occn)}


@pytest.mark.parametrize("N", [3, 8])
def test_springs_on_equilibrium_laws_extrapolate_in_dt(N):
    """With springs on, the stationary state of the scheme at dt = 0.01,
    0.005, 0.0025 differs from the equilibrium of Sec. 2.1 by a bias linear in
    dt, whose extrapolation to dt = 0 gives that equilibrium within 3 sigma:
    Z Poisson of mean N/N0 truncated at the capacity C = N (mean
    sum z p_z / sum p_z, p_z = lam^z / z!), spring positions uniform over the
    beads (share 2/N on the end beads), anchor offsets of variance N_s/3 and
    bonds of variance 1/3 per component.  The Euler-Maruyama bond-variance
    bias is positive (the discrete Ornstein-Uhlenbeck variance exceeds the
    continuous one by a factor 1 + k dt / 2 + O(dt^2)) and resolved."""
    M = 4096
    lam = N / N0
    p = np.array([lam ** z / math.factorial(z) for z in range(N + 1)])
    exact = {"Z": float((np.arange(N + 1) * p).sum() / p.sum()), "bond_var": 1.0 / 3.0,
             "offset_var": NS / 3.0, "end_share": 2.0 / N}
    dts = np.array([0.01, 0.005, 0.0025])
    res = [_stationary_averages(N, M, dt, seed=41 + N) for dt in dts]
    X = np.stack([np.ones(3), dts], axis=1)
    for key, want in exact.items():
        y = np.array([r[key][0] for r in res])
        s = np.array([r[key][1] for r in res])
        W = np.diag(1.0 / s ** 2)
        cov = np.linalg.inv(X.T @ W @ X)
        a, b = cov @ X.T @ W @ y
        chi2 = float((((y - (a + b * dts)) / s) ** 2).sum())
        assert stats.chi2.sf(chi2, 1) > 1e-3, (key, y, s, chi2)  # linear in dt
        assert abs(a - want) <= 3.0 * math.sqrt(cov[0, 0]), (key, a, math.sqrt(cov[0, 0]), want)
        if key == "bond_var":
            assert b > 5.0 * math.sqrt(cov[1, 1]), (b, math.sqrt(cov[1, 1]))


# --------------------------------------------- linear response (Sec. 2.3) ----

def test_step_strain_response_equals_green_kubo_with_virtual_stress():
    """The mean shear stress after a small step strain gamma, divided by gamma,
    equals <sigma_xy(t) [sigma_xy(0) + sigma^v_xy(0)]> (Green-Kubo form with the
    virtual stress, Sec. 2.3), not the plain stress autocorrelation alone.
    The strained and reference ensembles share their random streams (common
    random numbers); sigma_xy is odd in gamma, so the nonlinear error is
    O(gamma^3)."""
    N, M, gamma, T, TB = 8, 16384, 0.1, 120, 400
    kap = np.zeros((3, 3))
    kap[0, 1] = gamma / DT
    base = oracle.Ensemble([N] * M, seed=51).init()
    strained = oracle.Ensemble([N] * M, seed=51).init()
    s0 = base.stress()
    sb = np.concatenate([s0[None], base.run(TB, sample_every=1)], axis=0)  # sb[t] after t steps
    strained.step(kap)
    ss = np.concatenate([strained.stress()[None], strained.run(T - 1, sample_every=1)], axis=0)  # ss[t]: t+1 steps
    resp = (ss[:, :, 3] - sb[1:T + 1, :, 3]) / gamma
    x = sb[:, :, 3]
    y = sb[:, :, 3] + sb[:, :, 9]

    def gk(L, yy):
        per_chain = (x[L:] * yy[:TB + 1 - L]).mean(axis=0)
        return _batch_se(per_chain)

    results = []
    for L in [20, 40, 80, 119]:
        r_est, r_se = _batch_se(resp[L])
        g_full, g_se = gk(L + 1, y)   # response after L+1 steps of evolution
        g_plain, gp_se = gk(L + 1, x)
        results.append((L, r_est, g_full, g_plain))
        tol = 4.0 * math.hypot(r_se, g_se)
        assert abs(r_est - g_full) < tol + 0.02 * abs(g_full), (L, r_est, r_se, g_full, g_se, g_plain)
    # the virtual-stress term is needed: the plain autocorrelation misses the
    # response by many standard errors; lag 20 is where that gap (about 10 %)
    # is largest against the statistical error (z of 5 to 7 over seeds; the
    # response's error grows at longer lags)
    L = 20
    r_est, r_se = _batch_se(resp[L])
    g_plain, gp_se = gk(L + 1, x)
    assert abs(r_est - g_plain) > 4.0 * math.hypot(r_se, gp_se), results


def test_virtual_stress_contribution_at_zero_lag():
    """At t = 0 in equilibrium (the exact sampler, no dt bias) the two halves of
    the relative virtual-stress contribution (Sec. 4.1) have closed forms:
    the anchor offsets d_j are N(0, N_s/3) and independent of the bonds, so
    <sigma^v_xy (sigma + sigma^v)_xy> = (3/N_s)^2 <Z> (N_s/3)^2 = <Z> and
    <sigma_xy (sigma + sigma^v)_xy> = 9 (N-1) (1/3)^2 = N - 1; the same for yz
    and zx.  (For N = 8 the ratio <Z>/(N-1) = 0.286 is of the 25 % size the
    paper reports.)"""
    N, M = 8, 20000
    e = oracle.Ensemble([N] * M, seed=57).init()
    st = e.stress()
    Z = (e.S.reshape(M, N) >= 0).sum(axis=1)
    for c in range(3):
        sig, sv = st[:, 3 + c], st[:, 9 + c]
        num, num_se = _batch_se(sv * (sig + sv))
        den, den_se = _batch_se(sig * (sig + sv))
        assert abs(num - Z.mean()) < 4.0 * num_se, (c, num, Z.mean(), num_se)
        assert abs(den - (N - 1)) < 4.0 * den_se, (c, den, N - 1, den_se)
    lam = N / N0
    pz = np.array([math.exp(-lam) * lam**z / math.factorial(z) for z in range(N + 1)])
    assert Z.mean() == pytest.approx((pz * np.arange(N + 1)).sum() / pz.sum(), abs=4.0 * Z.std() / math.sqrt(M))


# -------------------------------------------------- multiple-tau correlator --

def test_multitau_constant_and_alternating_series():
    T = 1000
    C, cnt = oracle.multitau(np.full(T, 2.0), np.full(T, 3.0), levels=6, lags=16)
    ok = cnt > 0
    np.testing.assert_allclose(C[ok] / cnt[ok], 6.0, rtol=1e-14)
    x = (-1.0) ** np.arange(T)
    C, cnt = oracle.multitau(x, x, levels=4, lags=16)
    np.testing.assert_allclose(C[0] / cnt[0], (-1.0) ** np.arange(16), rtol=1e-14)
    assert np.all(C[1:] == 0.0)
    assert cnt[0, 0] == T and cnt[0, 15] == T - 15 and cnt[1, 0] == T // 2 and cnt[3, 3] == T // 8 - 3


def test_multitau_equals_block_mean_brute_force():
    rng = np.random.default_rng(2)
    T = 777
    x, y = rng.normal(size=T), rng.normal(size=T)
    C, cnt = oracle.multitau(x, y, levels=5, lags=16)
    for lvl in range(5):
        b = 2**lvl
        nb = T // b
        # level l of the pairwise-mean hierarchy has len_{l} = floor(len_{l-1}/2);
        # for these sizes it equals floor(T / 2^l)
        xb = x[: nb * b].reshape(nb, b).mean(axis=1)
        yb = y[: nb * b].reshape(nb, b).mean(axis=1)
        for k in range(16):
            want = float(np.dot(xb[k:], yb[: nb - k])) if nb > k else 0.0
            assert C[lvl, k] == pytest.approx(want, rel=1e-12, abs=1e-12)
            assert cnt[lvl, k] == max(0, nb - k)


# ------------------------------------------------------- structural facts ---

def test_run_equals_repeated_step_and_sharding_invariance():
    N = [5, 9, 12]
    a = oracle.Ensemble(N, seed=61).init()
    b = oracle.Ensemble(N, seed=61).init()
    kap = np.zeros((3, 3))
    kap[0, 1] = 0.3
    a.run(40, kappa=kap, keep_samples=False)
    for _ in range(40):
        b.step(kap)
    assert np.array_equal(a.R, b.R) and np.array_equal(a.A, b.A) and np.array_equal(a.S, b.S)
    # a chain's trajectory depends only on its global id, not on its neighbours
    c = oracle.Ensemble([12], chain_ids=[2], seed=61).init()
    c.run(40, kappa=kap, keep_samples=False)
    o = a.off[2]
    assert np.array_equal(c.R, a.R[o:o + 12]) and np.array_equal(c.S, a.S[o:o + 12])


def test_reconstruction_only_at_ends_and_capacity():
    e = oracle.Ensemble([6] * 500, seed=71).init()
    prev = e.S.copy()
    for _ in range(200):
        ev, _ = e.step(want_events=True)
        created = (ev & (oracle.EV_CREATE_FIRST | oracle.EV_CREATE_LAST)) != 0
        destroyed = (ev & oracle.EV_DESTROY) != 0
        assert np.all(prev[created] == -1)
        pos = e.S[created]
        assert np.all((pos == 0) | (pos == 5))
        assert np.all(e.S[destroyed] == -1)
        prev = e.S.copy()
    assert np.all(e.S < 6)


@pytest.mark.parametrize("rule", [0, 1], ids=["k_equals_c_minus_z", "k_equals_1"])
def test_destructions_per_window_stay_within_the_stored_log_capacity(rule):
    """A stored window logs the anchor of every destroyed spring, up to
    N + ceil(mu + 8 sqrt(mu)) + 16 entries per chain with mu = window 2 dt /
    (zeta_s N0).  The bound rests on two facts checked here on the oracle's
    own runs (Sec. 3.2 reconstruction step): each destruction ends a spring
    present at the window start or created in it, and the creations per chain
    and step have mean K 2 p_K <= 2 dt / (zeta_s N0) under either rule."""
    N, M, T = 16, 256, 2000
    o = oracle.Ensemble([N] * M, seed=41, construct_rule=rule).init()
    S0 = o.S.reshape(M, N).copy()
    created = np.zeros(M, dtype=np.int64)
    gone = np.zeros(M, dtype=np.int64)
    prev = S0
    for _ in range(T):
        o.step()
        cur = o.S.reshape(M, N)
        created += ((prev < 0) & (cur >= 0)).sum(axis=1)
        gone += ((prev >= 0) & (cur < 0)).sum(axis=1)
        prev = cur.copy()
    mu = T * 2.0 * o.dt / (o.zeta_s * o.n0)
    # conservation: springs at the end = at the start + created - destroyed
    assert np.array_equal((prev >= 0).sum(axis=1), (S0 >= 0).sum(axis=1) + created - gone)
    # the mean creation count is at most mu (5 standard errors of a Poisson mean)
    assert created.mean() <= mu + 5.0 * math.sqrt(mu / M)
    assert gone.max() <= N + math.ceil(mu + 8.0 * math.sqrt(mu)) + 16
