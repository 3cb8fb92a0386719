"""Pins of the oracle's discrete adjoint (derivative of a finite-time stress
with respect to the velocity gradient and the slip-spring strength N_s,
conditioned on the recorded events and normals).

Pinned against: central finite differences of the frozen-event forward map
(the same events and random normals, parameters perturbed), and the exact
mean slope d<sigma_xy(T)>/d(gdot) of the Euler-discretised Rouse chain
(springs off), derived independently below.
"""
import math

import numpy as np
import pytest

import oracle

DT = 0.01


def _kap(g=0.0, eps=0.0):
    k = np.zeros((3, 3))
    k[0, 1] = g
    k += np.diag([eps, -0.5 * eps, -0.5 * eps])
    return k


def _forced(N, M, St, T, kap, ns, seed):
    e = oracle.Ensemble([N] * M, seed=seed, ns=ns).init()
    for t in range(T):
        e.step_forced(St[t + 1], kap, ns=ns)
    return e


@pytest.fixture(scope="module")
def shear_window():
    N, M, T, g, ns, seed = 12, 24, 300, 0.3, 0.5, 5
    base = oracle.Ensemble([N] * M, seed=seed, ns=ns).init()
    Rt, At, St = base.run_record(T, _kap(g))
    return dict(N=N, M=M, T=T, g=g, ns=ns, seed=seed, base=base, Rt=Rt, At=At, St=St)


def test_frozen_event_replay_reproduces_the_run(shear_window):
    w = shear_window
    f = _forced(w["N"], w["M"], w["St"], w["T"], _kap(w["g"]), w["ns"], w["seed"])
    assert np.array_equal(f.R, w["base"].R)
    occ = w["base"].S >= 0
    assert np.array_equal(f.S, w["base"].S) and np.array_equal(f.A[occ], w["base"].A[occ])
    # the window has events of every kind
    St = w["St"]
    assert np.any((St[:-1] >= 0) & (St[1:] < 0)) and np.any((St[:-1] < 0) & (St[1:] >= 0))
    assert np.any((St[:-1] >= 0) & (St[1:] >= 0) & (St[:-1] != St[1:]))


def test_adjoint_equals_central_differences_shear(shear_window):
    w = shear_window
    gk, gns = w["base"].adjoint(w["Rt"], w["At"], w["St"], _kap(w["g"]), comp=3)
    h = 1e-4
    J = lambda e: e.stress()[:, 3]
    fd_g = (J(_forced(w["N"], w["M"], w["St"], w["T"], _kap(w["g"] + h), w["ns"], w["seed"]))
            - J(_forced(w["N"], w["M"], w["St"], w["T"], _kap(w["g"] - h), w["ns"], w["seed"]))) / (2 * h)
    fd_n = (J(_forced(w["N"], w["M"], w["St"], w["T"], _kap(w["g"]), w["ns"] + h, w["seed"]))
            - J(_forced(w["N"], w["M"], w["St"], w["T"], _kap(w["g"]), w["ns"] - h, w["seed"]))) / (2 * h)
    np.testing.assert_allclose(gk[:, 0, 1], fd_g, rtol=1e-8, atol=1e-8 * np.abs(fd_g).max())
    np.testing.assert_allclose(gns, fd_n, rtol=1e-6, atol=1e-6 * np.abs(fd_n).max())


def test_adjoint_equals_central_differences_elongation_normal_stress():
    N, M, T, eps, ns, seed = 9, 16, 200, 0.05, 0.5, 7
    base = oracle.Ensemble([N] * M, seed=seed, ns=ns).init()
    Rt, At, St = base.run_record(T, _kap(eps=eps))
    gk, _ = base.adjoint(Rt, At, St, _kap(eps=eps), comp=0)  # J = sigma_xx
    # directional derivative along diag(1, -1/2, -1/2)
    adj = gk[:, 0, 0] - 0.5 * gk[:, 1, 1] - 0.5 * gk[:, 2, 2]
    h = 1e-5
    J = lambda e: e.stress()[:, 0]
    fd = (J(_forced(N, M, St, T, _kap(eps=eps + h), ns, seed)) - J(_forced(N, M, St, T, _kap(eps=eps - h), ns, seed))) / (2 * h)
    np.testing.assert_allclose(adj, fd, rtol=1e-7, atol=1e-7 * np.abs(fd).max())
    # an off-diagonal kappa entry the flow does not use
    k2 = _kap(eps=eps)
    k2p, k2m = k2.copy(), k2.copy()
    k2p[2, 0] += h
    k2m[2, 0] -= h
    fd20 = (J(_forced(N, M, St, T, k2p, ns, seed)) - J(_forced(N, M, St, T, k2m, ns, seed))) / (2 * h)
    np.testing.assert_allclose(gk[:, 2, 0], fd20, rtol=1e-7, atol=1e-7 * max(np.abs(fd20).max(), 1e-12))


def rouse_shear_slope(N, dt, T):
    """d<sigma_xy(T)>/d(gdot) for the Euler-discretised Rouse chain started from
    bonds of variance 1/3: with b' = M b + dt gdot e_x b_y + noise,
    M = 1 - 3 dt B (B the bond Laplacian, eigenvalues lam_p = 4 sin^2(p pi/2N),
    rho_p = 1 - 3 dt lam_p), the slope is 3 dt sum_{m<T} sum_p rho_p^(2(T-m)-1)
    c_p(m) with c_p(m) = v_p + (1/3 - v_p) rho_p^(2m), v_p = 1/(3(1 - 1.5 dt lam_p))."""
    p = np.arange(1, N)
    lam = 4.0 * np.sin(p * np.pi / (2 * N)) ** 2
    rho = 1.0 - 3.0 * dt * lam
    v = 1.0 / (3.0 * (1.0 - 1.5 * dt * lam))
    tot = 0.0
    for m in range(T):
        c = v + (1.0 / 3.0 - v) * rho ** (2 * m)
        tot += float(np.sum(rho ** (2 * (T - m) - 1) * c))
    return 3.0 * dt * tot


def test_rouse_shear_slope_closed_form_matches_direct_covariance_recursion():
    # the closed form against an explicit covariance recursion in bond space
    N, dt, T = 6, DT, 150
    D = np.zeros((N - 1, N))
    for i in range(N - 1):
        D[i, i], D[i, i + 1] = -1.0, 1.0
    B = D @ D.T
    Mm = np.eye(N - 1) - 3 * dt * B
    C = np.eye(N - 1) / 3.0          # Cov(b_y(m))
    Ms = [np.linalg.matrix_power(Mm, k) for k in range(2 * T + 2)]
    slope = 0.0
    for m in range(T):
        slope += 3 * dt * np.trace(Ms[T - 1 - m] @ C @ Ms[T - m].T)
        C = Mm @ C @ Mm.T + 2 * dt * B
    assert rouse_shear_slope(N, dt, T) == pytest.approx(slope, rel=1e-12)


def test_adjoint_mean_equals_rouse_shear_slope():
    N, M, T, g = 8, 4096, 250, 0.01
    e = oracle.Ensemble([N] * M, seed=17, n0=1e30).init()  # springs off
    Rt, At, St = e.run_record(T, _kap(g))
    gk, _ = e.adjoint(Rt, At, St, _kap(g), comp=3)
    x = gk[:, 0, 1]
    b = np.array([c.mean() for c in np.array_split(x, 32)])
    est, se = b.mean(), b.std(ddof=1) / math.sqrt(32)
    want = rouse_shear_slope(N, DT, T)
    assert abs(est - want) < 4 * se, (est, want, se)
