// Setup, observable and reduction kernels of libssp: the equilibrium
// initial-state sampler, the multiple-tau correlator update, compensated
// chain/element reductions, and canonical state views.
#include "ssp_device.h"
#include "ssp_internal.h"

namespace ssp {

namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n, int per = kBlock) { return (unsigned)((n + per - 1) / per); }

// Neumaier compensated accumulation.
struct Neumaier {
    double s = 0.0, c = 0.0;
    __device__ void add(double x)
    {
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    __device__ double value() const { return s + c; }
};

// ---------------------------------------------------------------- init -----
// Equilibrium sampler (Sec. 3.1): R_0 = 0, bonds N(0, 1/3); Z from
// Poisson(N/N_0) truncated to 0..N; slots 0..Z-1 occupied with S uniform and
// A = R_S + N(0, N_s/3).  One thread per chain, FP64 arithmetic for both
// precisions (setup is not on the hot path); the FP32 state keeps the FP64
// value as hi + lo.
template <typename T>
__global__ void k_init(State st, ChainTables ct, int64_t M, Physics ph)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const int n = ct.n[k];
    const int64_t o = ct.off[k];
    const uint32_t gid = ct.gid[k];
    const double bsd = sqrt(1.0 / 3.0), asd = sqrt(ph.ns / 3.0);
    double R[3] = {0.0, 0.0, 0.0};
    auto put_r = [&](int i, const double* x) {
        if constexpr (sizeof(T) == 4) {
            float4 h, l;
            h.x = (float)x[0]; h.y = (float)x[1]; h.z = (float)x[2]; h.w = 0.f;
            l.x = (float)(x[0] - (double)h.x); l.y = (float)(x[1] - (double)h.y); l.z = (float)(x[2] - (double)h.z); l.w = 0.f;
            reinterpret_cast<float4*>(st.r0)[o + i] = h;
            reinterpret_cast<float4*>(st.r1)[o + i] = l;
        } else {
            reinterpret_cast<double4*>(st.r0)[o + i] = make_double4(x[0], x[1], x[2], 0.0);
        }
    };
    auto put_a = [&](int j, const double* x) {
        if constexpr (sizeof(T) == 4) {
            float4 h, l;
            h.x = (float)x[0]; h.y = (float)x[1]; h.z = (float)x[2]; h.w = 0.f;
            l.x = (float)(x[0] - (double)h.x); l.y = (float)(x[1] - (double)h.y); l.z = (float)(x[2] - (double)h.z); l.w = 0.f;
            reinterpret_cast<float4*>(st.a0)[o + j] = h;
            reinterpret_cast<float4*>(st.a1)[o + j] = l;
        } else {
            reinterpret_cast<double4*>(st.a0)[o + j] = make_double4(x[0], x[1], x[2], 0.0);
        }
    };
    put_r(0, R);
    for (int i = 0; i + 1 < n; ++i) {
        const v3<double> g = normals3_f64(draw(kInitBond, (uint32_t)i, gid, 0, ph.key0, ph.key1));
        R[0] += bsd * g.x;
        R[1] += bsd * g.y;
        R[2] += bsd * g.z;
        put_r(i + 1, R);
    }
    // truncated Poisson by inverse CDF
    const double lam = (double)n / ph.n0;
    const double u = u01<double>(draw(kInitZ, 0u, gid, 0, ph.key0, ph.key1).x);
    double pmf = exp(-lam), total = 0.0;
    for (int z = 0; z <= n; ++z) {
        if (z > 0) pmf = pmf * lam / (double)z;
        total += pmf;
    }
    int Z = n;
    pmf = exp(-lam);
    double cdf = 0.0;
    for (int z = 0; z <= n; ++z) {
        if (z > 0) pmf = pmf * lam / (double)z;
        cdf += pmf;
        if (u < cdf / total) {
            Z = z;
            break;
        }
    }
    for (int j = 0; j < n; ++j) {
        double A[3] = {0.0, 0.0, 0.0};
        int sj = -1;
        if (j < Z) {
            const uint32_t w = draw(kInitS, (uint32_t)j, gid, 0, ph.key0, ph.key1).x;
            sj = (int)(((uint64_t)w * (uint64_t)n) >> 32);
            // R_S: re-read the stored bead (hi + lo reproduces the FP64 value)
            double Rs[3];
            if constexpr (sizeof(T) == 4) {
                const float4 h = reinterpret_cast<const float4*>(st.r0)[o + sj];
                const float4 l = reinterpret_cast<const float4*>(st.r1)[o + sj];
                Rs[0] = (double)h.x + (double)l.x;
                Rs[1] = (double)h.y + (double)l.y;
                Rs[2] = (double)h.z + (double)l.z;
            } else {
                const double4 h = reinterpret_cast<const double4*>(st.r0)[o + sj];
                Rs[0] = h.x;
                Rs[1] = h.y;
                Rs[2] = h.z;
            }
            const v3<double> g = normals3_f64(draw(kInitAnchor, (uint32_t)j, gid, 0, ph.key0, ph.key1));
            A[0] = Rs[0] + asd * g.x;
            A[1] = Rs[1] + asd * g.y;
            A[2] = Rs[2] + asd * g.z;
        }
        put_a(j, A);
        st.s[o + j] = sj;
    }
}

__global__ void k_reset_ctrl(int64_t* ctrl, uint32_t* flags)
{
    const int t = threadIdx.x;
    if (t < kCtrlWords) ctrl[t] = 0;
    if (t == 0) *flags = 0u;
}

__global__ void k_zero(double* p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

__global__ void k_zero_ctrl_obs(int64_t* ctrl)
{
    if (threadIdx.x == 0) {
        ctrl[kCtrlCorrSamples] = 0;
        ctrl[kCtrlSeriesSamples] = 0;
    }
}

__device__ __forceinline__ int64_t samples_in(int64_t g0, int32_t n, int32_t every)
{
    return every > 0 ? (g0 + n) / every - g0 / every : 0;
}

__global__ void k_advance(int64_t* ctrl, int32_t n_steps, int32_t every, int64_t series_cap, uint32_t* flags)
{
    if (threadIdx.x != 0) return;
    const int64_t q = samples_in(ctrl[kCtrlSteps], n_steps, every);
    ctrl[kCtrlSteps] += n_steps;
    ctrl[kCtrlCorrSamples] += q;
    if (series_cap > 0 && ctrl[kCtrlSeriesSamples] + q > series_cap) atomicOr(flags, kFlagSeriesOverflow);
    ctrl[kCtrlSeriesSamples] += q;
}

// ------------------------------------------------------- correlator --------
// One 16-lane row per (chain, component) with lane k holding lag k at every
// level.  A new level-l value (x_l, y_l) shifts the y history of level l by
// one lane, adds x_l * y_l(n - k) to lane k, and is either parked as the
// first of a pair or averaged with the parked value into a level-(l+1) value.
// Histories start at zero, so unfilled lags add nothing; the number of
// products per lag is known from the sample count.  With the virtual-stress
// channel (V), x_v = sigma^v_ab(t) is paired with the same y history and
// block-averaged like x.
//
// The row is a DPP row (16 lanes): the history shift is row_shr:1 and the
// parked pair of level l is read with row_newbcast:l, so the level loop runs
// without LDS traffic (DPP controls are immediates: the level loop is fully
// unrolled).
__device__ __forceinline__ double row_shr1(double v)
{
    const int2 p = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_mov_dpp(p.x, 0x111, 0xf, 0xf, true),
                                                __builtin_amdgcn_mov_dpp(p.y, 0x111, 0xf, 0xf, true)));
}
template <int L> __device__ __forceinline__ double row_bcast(double v)
{
    const int2 p = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_mov_dpp(p.x, 0x150 + L, 0xf, 0xf, true),
                                                __builtin_amdgcn_mov_dpp(p.y, 0x150 + L, 0xf, 0xf, true)));
}
// row_bcast<l> for a level index that is a constant once the level loop is
// unrolled (the switch folds away).
__device__ __forceinline__ double row_bcast_level(double v, int l)
{
    switch (l) {
    case 0: return row_bcast<0>(v);
    case 1: return row_bcast<1>(v);
    case 2: return row_bcast<2>(v);
    case 3: return row_bcast<3>(v);
    case 4: return row_bcast<4>(v);
    case 5: return row_bcast<5>(v);
    case 6: return row_bcast<6>(v);
    case 7: return row_bcast<7>(v);
    case 8: return row_bcast<8>(v);
    case 9: return row_bcast<9>(v);
    case 10: return row_bcast<10>(v);
    case 11: return row_bcast<11>(v);
    case 12: return row_bcast<12>(v);
    case 13: return row_bcast<13>(v);
    case 14: return row_bcast<14>(v);
    default: return row_bcast<15>(v);
    }
}

template <bool V> __global__ void __launch_bounds__(kBlock) k_corr(CorrArgs a)
{
    const int64_t rows = 3 * a.n_chains;
    const int k = threadIdx.x & 15;
    const int64_t r = (int64_t)blockIdx.x * (kBlock / 16) + (threadIdx.x >> 4);
    const bool live = r < rows;
    const int64_t rr = live ? r : 0;
    const int64_t chain = rr / 3;
    const int comp = (int)(rr % 3);

    double yh[kMaxCorrLevels], C[kMaxCorrLevels], Cv[V ? kMaxCorrLevels : 1];
#pragma unroll
    for (int l = 0; l < kMaxCorrLevels; ++l) {
        yh[l] = (l < a.levels) ? a.hist[((int64_t)l * rows + rr) * 16 + k] : 0.0;
        C[l] = (l < a.levels) ? a.acc[((int64_t)l * rows + rr) * 16 + k] : 0.0;
        if constexpr (V) Cv[l] = (l < a.levels) ? a.acc_v[((int64_t)l * rows + rr) * 16 + k] : 0.0;
    }
    double px = a.pend[(rr * 16 + k) * 2 + 0];
    double py = a.pend[(rr * 16 + k) * 2 + 1];
    double pv = V ? a.pend_v[rr * 16 + k] : 0.0;

    const int64_t g0 = a.ctrl[kCtrlSteps];
    const int64_t s0 = a.ctrl[kCtrlCorrSamples];
    const int64_t Q = samples_in(g0, a.n_steps, a.sample_every);
    // the values of the next two samples are in flight while one is processed
    auto load = [&](int64_t q, double& x, double& v) {
        if (q < Q) {
            const double* smp = a.samples + (q * a.n_chains + chain) * kSampleValues;
            x = smp[3 + comp];
            v = smp[9 + comp];
        }
    };
    double nx0 = 0.0, nv0 = 0.0, nx1 = 0.0, nv1 = 0.0;
    load(0, nx0, nv0);
    load(1, nx1, nv1);
    for (int64_t q = 0; q < Q; ++q) {
        double xl = nx0;
        double xv = nv0;
        nx0 = nx1;
        nv0 = nv1;
        load(q + 2, nx1, nv1);
        double yl = xl + xv;
        const int64_t cnt1 = s0 + q + 1;  // 1-based index of this sample
        bool go = true;
#pragma unroll
        for (int l = 0; l < kMaxCorrLevels; ++l) {
            if (go && l < a.levels) {
                const double prev = row_shr1(yh[l]);
                yh[l] = (k == 0) ? yl : prev;
                C[l] += xl * yh[l];
                if constexpr (V) Cv[l] += xv * yh[l];
                if ((cnt1 >> l) & 1) {  // first of a pair at this level: park it
                    if (k == l) {
                        px = xl;
                        py = yl;
                        if constexpr (V) pv = xv;
                    }
                    go = false;
                } else {
                    const double qx = row_bcast_level(px, l);
                    const double qy = row_bcast_level(py, l);
                    xl = (qx + xl) * 0.5;
                    yl = (qy + yl) * 0.5;
                    if constexpr (V) xv = (row_bcast_level(pv, l) + xv) * 0.5;
                }
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int l = 0; l < kMaxCorrLevels; ++l) {
        if (l < a.levels) {
            a.hist[((int64_t)l * rows + r) * 16 + k] = yh[l];
            a.acc[((int64_t)l * rows + r) * 16 + k] = C[l];
            if constexpr (V) a.acc_v[((int64_t)l * rows + r) * 16 + k] = Cv[l];
        }
    }
    a.pend[(r * 16 + k) * 2 + 0] = px;
    a.pend[(r * 16 + k) * 2 + 1] = py;
    if constexpr (V) a.pend_v[r * 16 + k] = pv;
}

// Batch sums of the accumulators: out[b][l][k] = sum over the chains of batch
// b (contiguous, equal split) and the three components, Neumaier-compensated.
// One block per (batch, level); thread t takes lag t % 16 and every 16th row.
__global__ void __launch_bounds__(kBlock) k_corr_batches(const double* acc, int64_t n_chains, int32_t levels,
                                                         int32_t batches, double* out)
{
    const int b = blockIdx.x / levels;
    const int l = blockIdx.x % levels;
    const int64_t rows = 3 * n_chains;
    const int64_t c0 = n_chains * b / batches, c1 = n_chains * (b + 1) / batches;
    const int k = threadIdx.x & 15, sub = threadIdx.x >> 4;
    Neumaier nm;
    for (int64_t r = 3 * c0 + sub; r < 3 * c1; r += 16) nm.add(acc[((int64_t)l * rows + r) * 16 + k]);
    __shared__ double ps[kBlock], pc[kBlock];
    ps[threadIdx.x] = nm.s;
    pc[threadIdx.x] = nm.c;
    __syncthreads();
    if (sub == 0) {
        Neumaier tot;
        double cc = 0.0;
        for (int q = 0; q < 16; ++q) {
            tot.add(ps[q * 16 + k]);
            cc += pc[q * 16 + k];
        }
        out[((int64_t)b * levels + l) * 16 + k] = tot.value() + cc;
    }
}

// G = sum_b S_b / (3 M cnt); G_err = standard error of the batch means.
__global__ void k_corr_final(const double* bs, int64_t n_chains, int32_t levels, int32_t batches, int64_t samples,
                             double* G, double* G_err)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= levels * 16) return;
    const int l = t / 16, k = t % 16;
    const int64_t len = samples >> l;
    const int64_t cnt = len > k ? len - k : 0;
    if (cnt == 0) {
        G[t] = 0.0;
        G_err[t] = 0.0;
        return;
    }
    Neumaier tot;
    for (int b = 0; b < batches; ++b) tot.add(bs[((int64_t)b * levels + l) * 16 + k]);
    G[t] = tot.value() / (3.0 * (double)n_chains * (double)cnt);
    if (batches < 2) {
        G_err[t] = 0.0;
        return;
    }
    double mean = 0.0;
    for (int b = 0; b < batches; ++b) {
        const int64_t mb = n_chains * (b + 1) / batches - n_chains * b / batches;
        mean += bs[((int64_t)b * levels + l) * 16 + k] / (3.0 * (double)mb * (double)cnt);
    }
    mean /= batches;
    double var = 0.0;
    for (int b = 0; b < batches; ++b) {
        const int64_t mb = n_chains * (b + 1) / batches - n_chains * b / batches;
        const double v = bs[((int64_t)b * levels + l) * 16 + k] / (3.0 * (double)mb * (double)cnt) - mean;
        var += v * v;
    }
    G_err[t] = sqrt(var / (batches - 1) / batches);
}

// ---------------------------------------------------- element series -------
// series[e][t][c] = sum over the chains of element e of sigma_c (c < 6) for
// the samples of the launch just finished; Neumaier-compensated, fixed order.
__global__ void k_series(const double* samples, const int32_t* elem_off, int32_t E, int64_t M, int32_t n_steps,
                         int32_t every, int64_t q_cap, const int64_t* ctrl, double* series, int64_t cap)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t Q = samples_in(ctrl[kCtrlSteps], n_steps, every);
    if (t >= (int64_t)E * q_cap * 6) return;
    const int c = (int)(t % 6);
    const int64_t q = (t / 6) % q_cap;
    const int e = (int)(t / (6 * q_cap));
    if (q >= Q) return;
    const int64_t pos = ctrl[kCtrlSeriesSamples] + q;
    if (pos >= cap) return;
    Neumaier nm;
    for (int64_t k = elem_off[e]; k < elem_off[e + 1]; ++k) nm.add(samples[(q * M + k) * kSampleValues + c]);
    series[((int64_t)e * cap + pos) * 6 + c] = nm.value();
}

// ---------------------------------------------------------- stress ---------
template <typename T> __device__ __forceinline__ void load_pos(const State& st, int64_t i, bool anchor, double* x)
{
    if constexpr (sizeof(T) == 4) {
        const float4 h = reinterpret_cast<const float4*>(anchor ? st.a0 : st.r0)[i];
        const float4 l = reinterpret_cast<const float4*>(anchor ? st.a1 : st.r1)[i];
        x[0] = (double)h.x + (double)l.x;
        x[1] = (double)h.y + (double)l.y;
        x[2] = (double)h.z + (double)l.z;
    } else {
        const double4 h = reinterpret_cast<const double4*>(anchor ? st.a0 : st.r0)[i];
        x[0] = h.x;
        x[1] = h.y;
        x[2] = h.z;
    }
}

// Per-chain sigma and sigma^v of the current state (Sec. 2.1 stress,
// Appendix B virtual stress), FP64 from the canonical positions.
template <typename T> __global__ void k_stress(State st, ChainTables ct, int64_t M, double ns, double* out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const int n = ct.n[k];
    const int64_t o = ct.off[k];
    double p[12] = {0};
    double prev[3], cur[3];
    load_pos<T>(st, o, false, prev);
    for (int i = 1; i < n; ++i) {
        load_pos<T>(st, o + i, false, cur);
        const double bx = cur[0] - prev[0], by = cur[1] - prev[1], bz = cur[2] - prev[2];
        p[0] += 3.0 * bx * bx;
        p[1] += 3.0 * by * by;
        p[2] += 3.0 * bz * bz;
        p[3] += 3.0 * bx * by;
        p[4] += 3.0 * by * bz;
        p[5] += 3.0 * bz * bx;
        prev[0] = cur[0];
        prev[1] = cur[1];
        prev[2] = cur[2];
    }
    int z = 0;
    const double kss = 3.0 / ns;
    for (int j = 0; j < n; ++j) {
        const int sj = st.s[o + j];
        if (sj < 0) continue;
        ++z;
        double r[3], a[3];
        load_pos<T>(st, o + sj, false, r);
        load_pos<T>(st, o + j, true, a);
        const double dx = r[0] - a[0], dy = r[1] - a[1], dz = r[2] - a[2];
        p[6] += kss * dx * dx;
        p[7] += kss * dy * dy;
        p[8] += kss * dz * dz;
        p[9] += kss * dx * dy;
        p[10] += kss * dy * dz;
        p[11] += kss * dz * dx;
    }
    p[0] -= n;
    p[1] -= n;
    p[2] -= n;
    p[6] -= z;
    p[7] -= z;
    p[8] -= z;
    for (int q = 0; q < 12; ++q) out[k * 12 + q] = p[q];
}

template <typename T> __global__ void k_read_state(State st, int64_t total, double* R, double* A, int32_t* S)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    double x[3];
    load_pos<T>(st, i, false, x);
    R[3 * i] = x[0];
    R[3 * i + 1] = x[1];
    R[3 * i + 2] = x[2];
    load_pos<T>(st, i, true, x);
    A[3 * i] = x[0];
    A[3 * i + 1] = x[1];
    A[3 * i + 2] = x[2];
    S[i] = st.s[i];
}

template <typename T>
__global__ void k_write_state(State st, int64_t total, const double* R, const double* A, const int32_t* S)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    for (int which = 0; which < 2; ++which) {
        const double* src = which ? A : R;
        const double x0 = src[3 * i], x1 = src[3 * i + 1], x2 = src[3 * i + 2];
        if constexpr (sizeof(T) == 4) {
            float4 h, l;
            h.x = (float)x0; h.y = (float)x1; h.z = (float)x2; h.w = 0.f;
            l.x = (float)(x0 - (double)h.x); l.y = (float)(x1 - (double)h.y); l.z = (float)(x2 - (double)h.z); l.w = 0.f;
            reinterpret_cast<float4*>(which ? st.a0 : st.r0)[i] = h;
            reinterpret_cast<float4*>(which ? st.a1 : st.r1)[i] = l;
        } else {
            reinterpret_cast<double4*>(which ? st.a0 : st.r0)[i] = make_double4(x0, x1, x2, 0.0);
        }
    }
    st.s[i] = S[i];
}

template <typename T>
__global__ void k_rng_normals(uint32_t k0, uint32_t k1, uint32_t gid, int64_t step, int32_t bead, int32_t count,
                              double* out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    // the step-pair layout of the step kernel: NOISE pairs give (c, s, c) at
    // the even step 2k; the odd step takes the last sine and the NOISE2 pair
    const uint32_t idx = (uint32_t)(bead + t);
    const T c = normal_scale<T>(1.0);
    const uint4 x = draw(kNoise, idx, gid, step >> 1, k0, k1);
    T g[6];
    box_muller(x.x, x.y, c, g[0], g[1]);
    box_muller(x.z, x.w, c, g[2], g[3]);
    if (step & 1) {
        const uint4 y = draw(kNoise2, idx, gid, step >> 1, k0, k1);
        box_muller(y.x, y.y, c, g[4], g[5]);
    }
    const int o = (step & 1) ? 3 : 0;
    out[3 * t] = (double)g[o];
    out[3 * t + 1] = (double)g[o + 1];
    out[3 * t + 2] = (double)g[o + 2];
}

// ----------------------------------------------------- element means -------
// out[e][c] = (1 / M_e) sum over the chains k of element e of rows[k][c],
// c < ncols: the ensemble average of a per-chain quantity within one fluid
// element (the average of Sec. 2.1 over the element's chains).  One block per
// element; thread t takes the chains lo + t, lo + t + 256, ... with Neumaier
// sums per column, and thread c then adds the 256 partials of column c in
// thread order, so the result does not depend on timing.
constexpr int kMeanCols = 12;
__global__ void __launch_bounds__(kBlock) k_element_mean(const double* rows, int64_t stride, int32_t ncols,
                                                         const int32_t* elem_off, double* out)
{
    const int e = blockIdx.x;
    const int64_t lo = elem_off[e], hi = elem_off[e + 1];
    Neumaier nm[kMeanCols];
    for (int64_t k = lo + threadIdx.x; k < hi; k += kBlock)
        for (int c = 0; c < kMeanCols; ++c)
            if (c < ncols) nm[c].add(rows[k * stride + c]);
    __shared__ double ps[kMeanCols][kBlock], pc[kMeanCols][kBlock];
    for (int c = 0; c < kMeanCols; ++c) {
        ps[c][threadIdx.x] = nm[c].s;
        pc[c][threadIdx.x] = nm[c].c;
    }
    __syncthreads();
    if ((int)threadIdx.x < ncols) {
        const int c = threadIdx.x;
        Neumaier tot;
        double cc = 0.0;
        for (int t = 0; t < kBlock; ++t) {
            tot.add(ps[c][t]);
            cc += pc[c][t];
        }
        out[(int64_t)e * ncols + c] = (tot.value() + cc) / (double)(hi - lo);
    }
}

// ratio[t] = num[t] / den[t] on the multiple-tau grid where the lag has data
// and den != 0, NaN elsewhere (the relative contribution of the virtual
// stress to G(t), Sec. 4.1).
__global__ void k_grid_ratio(const double* num, const double* den, int32_t levels, int64_t samples, double* ratio)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= levels * 16) return;
    const int l = t / 16, k = t % 16;
    const int64_t len = samples >> l;
    ratio[t] = (len > k && den[t] != 0.0) ? num[t] / den[t] : __builtin_nan("");
}

}  // namespace

hipError_t launch_element_mean(const double* rows, int64_t stride, int32_t ncols, const int32_t* elem_off,
                               int32_t n_elements, double* out, hipStream_t s)
{
    if (ncols < 1 || ncols > kMeanCols || n_elements < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_element_mean, dim3((unsigned)n_elements), dim3(kBlock), 0, s, rows, stride, ncols, elem_off,
                       out);
    return hipGetLastError();
}

hipError_t launch_grid_ratio(const double* num, const double* den, int32_t levels, int64_t samples, double* ratio,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_grid_ratio, dim3(blocks_for(levels * 16)), dim3(kBlock), 0, s, num, den, levels, samples,
                       ratio);
    return hipGetLastError();
}

hipError_t launch_init(int precision, const State& st, const ChainTables& ct, int64_t M, Physics ph, hipStream_t s)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_init<float>, dim3(blocks_for(M, 64)), dim3(64), 0, s, st, ct, M, ph);
    else
        hipLaunchKernelGGL(k_init<double>, dim3(blocks_for(M, 64)), dim3(64), 0, s, st, ct, M, ph);
    return hipGetLastError();
}

hipError_t launch_reset_ctrl(int64_t* ctrl, uint32_t* flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_ctrl, dim3(1), dim3(64), 0, s, ctrl, flags);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(count)), dim3(kBlock), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_zero_ctrl_obs(int64_t* ctrl, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_ctrl_obs, dim3(1), dim3(64), 0, s, ctrl);
    return hipGetLastError();
}

hipError_t launch_advance(int64_t* ctrl, int32_t n_steps, int32_t sample_every, int64_t series_cap, uint32_t* flags,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ctrl, n_steps, sample_every, series_cap, flags);
    return hipGetLastError();
}

hipError_t launch_corr(const CorrArgs& a, hipStream_t s)
{
    const int64_t rows = 3 * a.n_chains;
    if (a.acc_v)
        hipLaunchKernelGGL(k_corr<true>, dim3(blocks_for(rows, kBlock / 16)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_corr<false>, dim3(blocks_for(rows, kBlock / 16)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_corr_batches(const double* acc, int64_t n_chains, int32_t levels, int32_t batches, double* out,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_corr_batches, dim3((unsigned)(batches * levels)), dim3(kBlock), 0, s, acc, n_chains, levels,
                       batches, out);
    return hipGetLastError();
}

hipError_t launch_corr_final(const double* batch_sums, int64_t n_chains, int32_t levels, int32_t batches,
                             int64_t corr_samples, double* G, double* G_err, hipStream_t s)
{
    hipLaunchKernelGGL(k_corr_final, dim3(blocks_for(levels * 16)), dim3(kBlock), 0, s, batch_sums, n_chains, levels,
                       batches, corr_samples, G, G_err);
    return hipGetLastError();
}

hipError_t launch_series(const double* samples, const int32_t* elem_off, int32_t n_elements, int64_t n_chains,
                         int32_t n_steps, int32_t sample_every, int64_t q_cap, const int64_t* ctrl, double* series,
                         int64_t series_cap, hipStream_t s)
{
    const int64_t threads = (int64_t)n_elements * q_cap * 6;
    hipLaunchKernelGGL(k_series, dim3(blocks_for(threads)), dim3(kBlock), 0, s, samples, elem_off, n_elements,
                       n_chains, n_steps, sample_every, q_cap, ctrl, series, series_cap);
    return hipGetLastError();
}

hipError_t launch_stress(int precision, const State& st, const ChainTables& ct, int64_t M, double ns, double* out,
                         hipStream_t s)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_stress<float>, dim3(blocks_for(M)), dim3(kBlock), 0, s, st, ct, M, ns, out);
    else
        hipLaunchKernelGGL(k_stress<double>, dim3(blocks_for(M)), dim3(kBlock), 0, s, st, ct, M, ns, out);
    return hipGetLastError();
}

hipError_t launch_read_state(int precision, const State& st, int64_t total, double* R, double* A, int32_t* S,
                             hipStream_t s)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_read_state<float>, dim3(blocks_for(total)), dim3(kBlock), 0, s, st, total, R, A, S);
    else
        hipLaunchKernelGGL(k_read_state<double>, dim3(blocks_for(total)), dim3(kBlock), 0, s, st, total, R, A, S);
    return hipGetLastError();
}

hipError_t launch_write_state(int precision, const State& st, int64_t total, const double* R, const double* A,
                              const int32_t* S, hipStream_t s)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_write_state<float>, dim3(blocks_for(total)), dim3(kBlock), 0, s, st, total, R, A, S);
    else
        hipLaunchKernelGGL(k_write_state<double>, dim3(blocks_for(total)), dim3(kBlock), 0, s, st, total, R, A, S);
    return hipGetLastError();
}

hipError_t launch_rng_normals(int precision, uint32_t key0, uint32_t key1, uint32_t gid, int64_t step, int32_t bead,
                              int32_t count, double* out, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (precision == 0)
        hipLaunchKernelGGL(k_rng_normals<float>, dim3(blocks_for(count)), dim3(kBlock), 0, s, key0, key1, gid, step,
                           bead, count, out);
    else
        hipLaunchKernelGGL(k_rng_normals<double>, dim3(blocks_for(count)), dim3(kBlock), 0, s, key0, key1, gid, step,
                           bead, count, out);
    return hipGetLastError();
}

}  // namespace ssp
