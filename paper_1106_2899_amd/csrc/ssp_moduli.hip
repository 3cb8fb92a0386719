// Linear viscoelasticity from the relaxation modulus G(t) that the
// multiple-tau correlator produces (the relations of Sec. 4.1):
//   G'(w)   = w int_0^inf G(t) sin(w t) dt,   G''(w) = w int_0^inf G(t) cos(w t) dt,
//   eta_0   = int_0^inf G(t) dt,              1/tau_d = -lim ln G(t) / t,
// |eta*(w)| = |G'(w) + i G''(w)| / w.
//
// The paper integrates with the trapezoidal rule.  The grid here is the
// log-spaced multiple-tau one (level 0 lags 0..15, level l >= 1 lags 8..15 of
// block length 2^l samples, lags with data only), whose spacing outgrows the
// period of sin(w t) while G is still large; so G is taken piecewise linear
// between grid points (the trapezoid's own model of the integrand) and that
// interpolant is integrated exactly against sin and cos, in forms where no
// two large terms cancel.  eta_0 is the plain trapezoidal sum.  The integrals
// stop at the last point with data.  tau_d is -1 over the least-squares slope
// of ln G against t on a window [t_lo, t_hi] of the tail (points with G > 0).
#include <math.h>

#include "ssp_internal.h"

namespace ssp {

namespace {

// sin h - h cos h: Taylor series sum_k (-1)^(k+1) 2k h^(2k+1) / (2k+1)! (k = 1..8)
// for |h| < 1/2, where the difference cancels; directly otherwise.
__device__ double sin_minus_hcos(double h)
{
    if (fabs(h) >= 0.5) return sin(h) - h * cos(h);
    double s = 0.0, p = h * h * h, fact = 6.0;  // h^(2k+1), (2k+1)!
    const double h2 = h * h;
    for (int k = 1; k <= 8; ++k) {
        s += ((k & 1) ? 1.0 : -1.0) * (2.0 * k) * p / fact;
        p *= h2;
        fact *= (2.0 * k + 2.0) * (2.0 * k + 3.0);
    }
    return s;
}

// The point (t, G) of the grid with index p in increasing t, or false past the end.
struct Grid {
    const double* G;
    int levels;
    int64_t samples;
    double sample_dt;
    __device__ bool point(int p, double& t, double& g) const
    {
        // level 0 holds points 0..15, every further level 8 points
        const int l = p < 16 ? 0 : 1 + (p - 16) / 8;
        const int k = p < 16 ? p : 8 + (p - 16) % 8;
        if (l >= levels || (samples >> l) <= k) return false;
        t = (double)k * ldexp(1.0, l) * sample_dt;
        g = G[l * 16 + k];
        return true;
    }
};

__global__ void k_moduli(Grid grid, const double* omega, int32_t n_omega, double t_lo, double t_hi, double* moduli,
                         double* scalars)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_omega) {
        const double w = omega[j];
        double gp = 0.0, gpp = 0.0, ta, ga, tb, gb;
        if (grid.point(0, ta, ga)) {
            for (int p = 1; grid.point(p, tb, gb); ++p) {
                const double m = (gb - ga) / (tb - ta);
                const double h = 0.5 * w * (tb - ta);
                const double c = 0.5 * w * (ta + tb);
                const double sh = sin(h), s3 = sin_minus_hcos(h);
                double sc, cc;
                sincos(c, &sc, &cc);
                gp += ga * 2.0 * sc * sh + m * (2.0 / w) * (cc * s3 + h * sc * sh);
                gpp += ga * 2.0 * cc * sh + m * (2.0 / w) * (h * cc * sh - sc * s3);
                ta = tb;
                ga = gb;
            }
        }
        moduli[3 * j] = gp;
        moduli[3 * j + 1] = gpp;
        moduli[3 * j + 2] = sqrt(gp * gp + gpp * gpp) / w;
    }
    if (j == 0) {
        double eta = 0.0, ta, ga, tb, gb;
        if (grid.point(0, ta, ga))
            for (int p = 1; grid.point(p, tb, gb); ++p) {
                eta += 0.5 * (tb - ta) * (ga + gb);
                ta = tb;
                ga = gb;
            }
        // least-squares slope of ln G on the window, two passes
        int n = 0;
        double sx = 0.0, sy = 0.0, t, g;
        for (int p = 0; grid.point(p, t, g); ++p)
            if (t >= t_lo && t <= t_hi && g > 0.0) {
                ++n;
                sx += t;
                sy += log(g);
            }
        double tau = NAN;
        if (n >= 2) {
            const double mx = sx / n, my = sy / n;
            double sxx = 0.0, sxy = 0.0;
            for (int p = 0; grid.point(p, t, g); ++p)
                if (t >= t_lo && t <= t_hi && g > 0.0) {
                    sxx += (t - mx) * (t - mx);
                    sxy += (t - mx) * (log(g) - my);
                }
            if (sxx > 0.0 && sxy / sxx < 0.0) tau = -sxx / sxy;
        }
        scalars[0] = eta;
        scalars[1] = tau;
    }
}

}  // namespace

hipError_t launch_moduli(const double* G, int32_t levels, int64_t samples, double sample_dt, const double* omega,
                         int32_t n_omega, double t_lo, double t_hi, double* moduli, double* scalars, hipStream_t s)
{
    const Grid grid{G, levels, samples, sample_dt};
    const int threads = 128;
    const int blocks = n_omega > 0 ? (n_omega + threads - 1) / threads : 1;
    hipLaunchKernelGGL(k_moduli, dim3(blocks), dim3(threads), 0, s, grid, omega, n_omega, t_lo, t_hi, moduli, scalars);
    return hipGetLastError();
}

}  // namespace ssp
