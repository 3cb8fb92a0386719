"""Linear viscoelasticity from a relaxation modulus on the multiple-tau grid.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64 Python,
written from the definitions of Sec. 4.1:

    G'(w)   = w * integral_0^inf G(t) sin(w t) dt      (storage modulus)
    G''(w)  = w * integral_0^inf G(t) cos(w t) dt      (loss modulus)
    eta_0   = integral_0^inf G(t) dt                   (zero-shear viscosity)
    1/tau_d = -lim_{t->inf} ln G(t) / t                (longest relaxation time)

The paper integrates with the trapezoidal rule.  On the log-spaced
multiple-tau grid the spacing outgrows the period of sin(w t) while G is
still large, so the rule is applied to G alone: G is taken piecewise linear
between the grid points (the trapezoid's own model of the integrand), and
that interpolant is integrated exactly against sin and cos (Filon's idea).  For eta_0 this
is the plain trapezoidal sum.  The integrals stop at the last grid point
with data.  |eta*(w)| = sqrt(G'^2 + G''^2) / w.  The limit defining tau_d is
the least-squares slope of ln G(t) against t over a window [t_lo, t_hi] of
the tail (points with G > 0).
"""
from __future__ import annotations

import math

import numpy as np


def multitau_grid(levels: int, samples: int, sample_dt: float):
    """Lag times and flat (level * 16 + lag) indices of the multiple-tau grid:
    level 0 lags 0..15, level l >= 1 lags 8..15 (block length 2^l samples),
    keeping the lags that have at least one product after `samples` samples."""
    t, idx = [], []
    for lvl in range(levels):
        n = samples >> lvl
        for k in range(0 if lvl == 0 else 8, 16):
            if n > k:
                t.append(k * (2 ** lvl) * sample_dt)
                idx.append(lvl * 16 + k)
    return np.array(t), np.array(idx, dtype=np.int64)


def _s3(h):
    """sin h - h cos h, by its Taylor series sum_k (-1)^(k+1) 2k h^(2k+1)/(2k+1)!
    for |h| < 1/2 (where the difference would cancel), directly otherwise."""
    if abs(h) >= 0.5:
        return math.sin(h) - h * math.cos(h)
    s, term = 0.0, None
    for k in range(1, 9):
        term = (-1) ** (k + 1) * 2 * k * h ** (2 * k + 1) / math.factorial(2 * k + 1)
        s += term
    return s


def segment_terms(a, b, ga, gb, w):
    """Exact w * int_a^b G(t) (sin w t, cos w t) dt for G linear from ga to gb:
    with m the slope, h = w (b - a) / 2, c = w (a + b) / 2,
      w int G sin = ga * 2 sin c sin h + m (2/w) [cos c (sin h - h cos h) + h sin c sin h]
      w int G cos = ga * 2 cos c sin h + m (2/w) [h cos c sin h - sin c (sin h - h cos h)],
    forms in which no two large terms cancel (the integrated-by-parts form
    loses ~(w t)^-2 of its digits at small w)."""
    m = (gb - ga) / (b - a)
    h = 0.5 * w * (b - a)
    c = 0.5 * w * (a + b)
    sh, s3 = math.sin(h), _s3(h)
    sp = ga * 2.0 * math.sin(c) * sh + m * (2.0 / w) * (math.cos(c) * s3 + h * math.sin(c) * sh)
    cp = ga * 2.0 * math.cos(c) * sh + m * (2.0 / w) * (h * math.cos(c) * sh - math.sin(c) * s3)
    return sp, cp


def dynamic_moduli(t, G, omega):
    """[len(omega)][3]: G', G'', |eta*|, G linear between grid points and
    integrated exactly against sin and cos segment by segment."""
    out = np.zeros((len(omega), 3))
    for j, w in enumerate(omega):
        gp = gpp = 0.0
        for i in range(len(t) - 1):
            sp, cp = segment_terms(t[i], t[i + 1], G[i], G[i + 1], w)
            gp += sp
            gpp += cp
        out[j] = (gp, gpp, math.sqrt(gp * gp + gpp * gpp) / w)
    return out


def moduli_error_scale(t, G, omega):
    """[len(omega)][2]: sum over segments of |each product in segment_terms|,
    the magnitude that bounds the rounding error of the sums."""
    out = np.zeros((len(omega), 2))
    for j, w in enumerate(omega):
        for i in range(len(t) - 1):
            a, b, ga, gb = t[i], t[i + 1], G[i], G[i + 1]
            m = (gb - ga) / (b - a)
            h = 0.5 * w * (b - a)
            scale = abs(ga) * 2.0 * abs(math.sin(h)) + abs(m) * (2.0 / w) * (abs(_s3(h)) + abs(h * math.sin(h)))
            out[j] += scale
    return out


def zero_shear_viscosity(t, G):
    s = 0.0
    for i in range(len(t) - 1):
        s += 0.5 * (t[i + 1] - t[i]) * (G[i] + G[i + 1])
    return s


def longest_relaxation_time(t, G, t_lo, t_hi):
    """-1 / (least-squares slope of ln G over the window); nan when fewer than
    two points qualify or the slope is not negative."""
    xs = [t[i] for i in range(len(t)) if t_lo <= t[i] <= t_hi and G[i] > 0.0]
    ys = [math.log(G[i]) for i in range(len(t)) if t_lo <= t[i] <= t_hi and G[i] > 0.0]
    n = len(xs)
    if n < 2:
        return float("nan")
    mx, my = sum(xs) / n, sum(ys) / n
    sxx = sum((x - mx) ** 2 for x in xs)
    sxy = sum((x - mx) * (y - my) for x, y in zip(xs, ys))
    if sxx == 0.0 or sxy / sxx >= 0.0:
        return float("nan")
    return -sxx / sxy
