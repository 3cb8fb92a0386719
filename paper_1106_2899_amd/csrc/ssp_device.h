// Device helpers for the slip-spring kernels: counter-based random numbers,
// small 3-vectors, cross-lane exchange and compensated FP32 accumulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ssp_internal.h"

namespace ssp {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies by the published multipliers, each round mixing the
// high halves with the other two counter words and the round key; the key is
// bumped by the published Weyl constants between rounds.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        // three-input xor in one v_bitop3_b32 (truth table 0x96)
        c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(m1 >> 32), c.y, k0, 0x96), (uint32_t)m1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), c.w, k1, 0x96), (uint32_t)m0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Counter (index, chain id, step lo, step hi | purpose << 24), for steps below
// 2^56.  The first round multiplies only the index and the step's low word,
// so its two products are the same for every purpose at a given step and
// index: a step's draws share them.
__device__ __forceinline__ uint4 draw(uint32_t purpose, uint32_t index, uint32_t gid, int64_t step, uint32_t k0,
                                      uint32_t k1)
{
    return philox(make_uint4(index, gid, (uint32_t)(uint64_t)step, (uint32_t)((uint64_t)step >> 32) | (purpose << 24)),
                  k0, k1);
}

// A value that every lane of the wavefront holds, moved to a scalar register
// (frees VGPRs; only valid when the caller knows the value is wave-uniform).
__device__ __forceinline__ float wave_uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double wave_uniform(double v)
{
    const int2 p = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readfirstlane(p.x), __builtin_amdgcn_readfirstlane(p.y)));
}
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int64_t wave_uniform(int64_t v)
{
    const int2 p = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(int64_t, make_int2(__builtin_amdgcn_readfirstlane(p.x), __builtin_amdgcn_readfirstlane(p.y)));
}

// u = ((w >> 9) + 1/2) 2^-23: 23 random bits, exactly representable in
// binary32 and binary64, never 0 or 1.
template <typename T> __device__ __forceinline__ T u01(uint32_t w);
template <> __device__ __forceinline__ float u01<float>(uint32_t w)
{
    // 0x3F800000 | (w >> 9) is 1 + (w >> 9) 2^-23 in one v_alignbit_b32;
    // subtracting 1 - 2^-24 is exact (both operands lie in [1/2, 2]).
    const float one_plus = __builtin_bit_cast(float, __builtin_amdgcn_alignbit(0x7Fu, w, 9u));
    return one_plus - (1.0f - 0x1p-24f);
}
template <> __device__ __forceinline__ double u01<double>(uint32_t w)
{
    return __fma_rn((double)(w >> 9), 0x1p-23, 0x1p-24);
}

template <typename T> struct v3 {
    T x, y, z;
};
template <typename T> __device__ __forceinline__ v3<T> mk(T x, T y, T z) { return v3<T>{x, y, z}; }
template <typename T> __device__ __forceinline__ v3<T> operator+(v3<T> a, v3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T> __device__ __forceinline__ v3<T> operator-(v3<T> a, v3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T> __device__ __forceinline__ v3<T> operator*(T s, v3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T> __device__ __forceinline__ v3<T> operator-(v3<T> a) { return {-a.x, -a.y, -a.z}; }
template <typename T> __device__ __forceinline__ T dot(v3<T> a, v3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T> __device__ __forceinline__ v3<T> zero3() { return {T(0), T(0), T(0)}; }
template <typename T> __device__ __forceinline__ v3<T> sel(bool c, v3<T> a, v3<T> b) { return c ? a : b; }

// Box-Muller normals from four words, scaled by sigma: sigma (r1 cos t1,
// r1 sin t1, r2 cos t2), r = sqrt(-2 ln u_a), t = 2 pi u_b.  The scale enters
// under the root: c = -2 sigma^2 (FP64, natural log) or -2 ln2 sigma^2 (FP32,
// base-2 log).
__device__ __forceinline__ v3<float> normals3_f32_scaled(uint4 w, float c)
{
    const float u0 = u01<float>(w.x), u1 = u01<float>(w.y), u2 = u01<float>(w.z), u3 = u01<float>(w.w);
    // the hardware sine/cosine take revolutions
    const float r1 = __builtin_amdgcn_sqrtf(c * __builtin_amdgcn_logf(u0));
    const float r2 = __builtin_amdgcn_sqrtf(c * __builtin_amdgcn_logf(u2));
    return {r1 * __builtin_amdgcn_cosf(u1), r1 * __builtin_amdgcn_sinf(u1), r2 * __builtin_amdgcn_cosf(u3)};
}
__device__ __forceinline__ v3<double> normals3_f64_scaled(uint4 w, double c)
{
    const double u0 = u01<double>(w.x), u1 = u01<double>(w.y), u2 = u01<double>(w.z), u3 = u01<double>(w.w);
    const double r1 = sqrt(c * log(u0));
    const double r2 = sqrt(c * log(u2));
    // sin/cos of pi (2u): 2u is exact, so no range reduction by 2 pi
    double s1, c1;
    sincospi(2.0 * u1, &s1, &c1);
    return {r1 * c1, r1 * s1, r2 * cospi(2.0 * u3)};
}
__device__ __forceinline__ v3<float> normals3_f32(uint4 w) { return normals3_f32_scaled(w, -1.38629436111989061883f); }
__device__ __forceinline__ v3<double> normals3_f64(uint4 w) { return normals3_f64_scaled(w, -2.0); }

// One Box-Muller pair scaled by sigma, (r cos t, r sin t) with
// r = sigma sqrt(-2 ln u_a), t = 2 pi u_b; c as for normals3_*_scaled.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float c, float& cs, float& sn)
{
    const float r = __builtin_amdgcn_sqrtf(c * __builtin_amdgcn_logf(u01<float>(wa)));
    const float t = u01<float>(wb);  // revolutions
    cs = r * __builtin_amdgcn_cosf(t);
    sn = r * __builtin_amdgcn_sinf(t);
}
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double c, double& cs, double& sn)
{
    const double r = sqrt(c * log(u01<double>(wa)));
    double s, co;
    sincospi(2.0 * u01<double>(wb), &s, &co);
    cs = r * co;
    sn = r * s;
}

// The root constant c of normals3_*_scaled for standard deviation sigma.
template <typename T> __device__ __forceinline__ T normal_scale(double sigma);
template <> __device__ __forceinline__ float normal_scale<float>(double sigma) { return (float)(-2.0 * M_LN2 * sigma * sigma); }
template <> __device__ __forceinline__ double normal_scale<double>(double sigma) { return -2.0 * sigma * sigma; }

template <typename T> __device__ __forceinline__ v3<T> normals3_scaled(uint4 w, T c);
template <> __device__ __forceinline__ v3<float> normals3_scaled<float>(uint4 w, float c) { return normals3_f32_scaled(w, c); }
template <> __device__ __forceinline__ v3<double> normals3_scaled<double>(uint4 w, double c) { return normals3_f64_scaled(w, c); }

template <typename T> __device__ __forceinline__ v3<T> normals3(uint4 w);
template <> __device__ __forceinline__ v3<float> normals3<float>(uint4 w) { return normals3_f32(w); }
template <> __device__ __forceinline__ v3<double> normals3<double>(uint4 w) { return normals3_f64(w); }

// Glauber hop probability min{h [1 - tanh(q y)], 1/2}, written as
// min{2h / (1 + e^{2 q y}), 1/2}, which stays accurate when tanh -> 1.  The
// caller passes h2 = 2h and e2q = 2q (FP64) or 2q log2(e) (FP32, base-2 exp).
__device__ __forceinline__ float glauber(float y, float e2q, float h2)
{
    return fminf(h2 * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(e2q * y)), 0.5f);
}
__device__ __forceinline__ double glauber(double y, double e2q, double h2) { return fmin(h2 / (1.0 + exp(e2q * y)), 0.5); }

template <typename T> __device__ __forceinline__ T glauber_exp_scale(double q);
template <> __device__ __forceinline__ float glauber_exp_scale<float>(double q) { return (float)(2.0 * q * M_LOG2E); }
template <> __device__ __forceinline__ double glauber_exp_scale<double>(double q) { return 2.0 * q; }

__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T> __device__ __forceinline__ v3<T> fma3(T s, v3<T> a, v3<T> b)
{
    return {fmat(s, a.x, b.x), fmat(s, a.y, b.y), fmat(s, a.z, b.z)};
}
// b + M r for a row-major 3x3 M, as fused multiply-adds.
template <typename T> __device__ __forceinline__ v3<T> fma_mat3(const T* m, v3<T> r, v3<T> b)
{
    return {fmat(m[0], r.x, fmat(m[1], r.y, fmat(m[2], r.z, b.x))),
            fmat(m[3], r.x, fmat(m[4], r.y, fmat(m[5], r.z, b.y))),
            fmat(m[6], r.x, fmat(m[7], r.y, fmat(m[8], r.z, b.z)))};
}

// Neighbour exchange across the whole wavefront with DPP: lane i receives
// lane i+1 (from_next, wave_shl:1) or lane i-1 (from_prev, wave_shr:1); the
// lane without a source receives 0 (bound_ctrl), which also lets the compiler
// fold the shift into the instruction that consumes it.
__device__ __forceinline__ int dpp_next_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_prev_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ float from_next(float v) { return __builtin_bit_cast(float, dpp_next_i(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ float from_prev(float v) { return __builtin_bit_cast(float, dpp_prev_i(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ double from_next(double v)
{
    const int2 p = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(dpp_next_i(p.x), dpp_next_i(p.y)));
}
__device__ __forceinline__ double from_prev(double v)
{
    const int2 p = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(dpp_prev_i(p.x), dpp_prev_i(p.y)));
}
template <typename T> __device__ __forceinline__ v3<T> from_next3(v3<T> v) { return {from_next(v.x), from_next(v.y), from_next(v.z)}; }
template <typename T> __device__ __forceinline__ v3<T> from_prev3(v3<T> v) { return {from_prev(v.x), from_prev(v.y), from_prev(v.z)}; }

// Cross-lane reads (ds_bpermute).
__device__ __forceinline__ float lane_read(float v, int src) { return __shfl(v, src, kWaveSize); }
__device__ __forceinline__ double lane_read(double v, int src) { return __shfl(v, src, kWaveSize); }
__device__ __forceinline__ int lane_read(int v, int src) { return __shfl(v, src, kWaveSize); }
template <typename T> __device__ __forceinline__ v3<T> lane_read3(v3<T> v, int src)
{
    return {lane_read(v.x, src), lane_read(v.y, src), lane_read(v.z, src)};
}

// (hi, lo) accumulation: adds inc to the value hi + lo, keeping the rounding
// error of the sum in lo (Kahan/Fast2Sum form; exact whenever |hi| >= |inc + lo|).
__device__ __forceinline__ void cadd(float& hi, float& lo, float inc)
{
    const float y = inc + lo;
    const float s = hi + y;
    lo = y - (s - hi);
    hi = s;
}
__device__ __forceinline__ void cadd3(v3<float>& hi, v3<float>& lo, v3<float> inc)
{
    cadd(hi.x, lo.x, inc.x);
    cadd(hi.y, lo.y, inc.y);
    cadd(hi.z, lo.z, inc.z);
}

// Test of the bits `bits` of a wave-uniform mask, as a scalar branch
// condition of its own: the empty asm statement stops the compiler from
// sharing one test between several branches, which it would otherwise keep as
// a 64-bit lane mask in scalar registers (and spill them).
__device__ __forceinline__ bool any_bits(uint32_t mask, uint32_t bits)
{
    asm volatile("" : "+s"(mask));
    return (mask & bits) != 0u;
}

// Error-free transformations (Knuth's TwoSum; the FMA form of the exact
// product): s + t = a + b and p + e = a b exactly in binary32.  Contraction is
// off so that the compiler cannot fuse a product into a later sum.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& t)
{
#pragma clang fp contract(off)
    s = a + b;
    const float bb = s - a;
    t = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e)
{
#pragma clang fp contract(off)
    p = a * b;
    e = __builtin_fmaf(a, b, -p);
}

// Row r of the affine flow increment K (h + l) of a compensated position
// (h, l), K = dt kappa, as big + small: big is the binary32 sum of the
// products K_rc h_c, small carries the rounding errors of those products and
// sums and the products with the low part, K_rc l_c.  `mask` marks the
// entries of K that are nonzero anywhere in the wavefront (a wave-uniform
// value: the tests are uniform branches).
template <int R>
__device__ __forceinline__ void flow_row(const float* K, uint32_t mask, v3<float> h, v3<float> l, float& big,
                                         float& small)
{
#pragma clang fp contract(off)
    const float hc[3] = {h.x, h.y, h.z};
    const float lc[3] = {l.x, l.y, l.z};
    big = 0.0f;
    small = 0.0f;
    bool first = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (any_bits(mask, 1u << (3 * R + c))) {
            float p, e;
            two_prod(K[3 * R + c], hc[c], p, e);
            small = small + __builtin_fmaf(K[3 * R + c], lc[c], e);
            if (first) {
                big = p;
                first = false;
            } else {
                float s, t;
                two_sum(big, p, s, t);
                big = s;
                small = small + t;
            }
        }
    }
}

// K (h + l) of a compensated position (h, l) for the entries of K marked in
// `mask` (wave-uniform; the others are known to be zero in every lane), as
// fused multiply-adds in row order, h before l for each entry.  The empty asm
// statement keeps each test a scalar branch: without it the compiler computes
// all nine products and picks the results with vector selects, which costs
// more than the products a typical kappa needs.
__device__ __forceinline__ v3<float> masked_mat3(const float* K, uint32_t mask, v3<float> h, v3<float> l)
{
    const float hc[3] = {h.x, h.y, h.z};
    const float lc[3] = {l.x, l.y, l.z};
    float r[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (any_bits(mask, 1u << (3 * a + c))) {
                r[a] = __builtin_fmaf(K[3 * a + c], lc[c], __builtin_fmaf(K[3 * a + c], hc[c], r[a]));
                asm volatile("" : "+v"(r[a]));
            }
    return {r[0], r[1], r[2]};
}

// (h, l) += big + inc, with big added error-free: the rounding of h + big is
// carried into l before the renormalisation.
__device__ __forceinline__ void cadd_big(float& hi, float& lo, float big, float inc)
{
#pragma clang fp contract(off)
    float s, t;
    two_sum(hi, big, s, t);
    const float y = (inc + t) + lo;
    hi = s + y;
    lo = y - (hi - s);
}

// One component of the error-free move of a stretched chain:
// (h, l) += (big + small) + c lap + rest, where big + small is the flow term
// (flow_row), c lap the bond force (lap from the compensated positions) and
// rest the noise and slip-spring force.  The bond force is split exactly
// (two_prod) and its large part joined to big by an exact TwoSum.
__device__ __forceinline__ void cadd_force(float& hi, float& lo, float big, float small, float c, float lap,
                                           float rest)
{
#pragma clang fp contract(off)
    float pf, ef, tot, t;
    two_prod(c, lap, pf, ef);
    two_sum(big, pf, tot, t);
    cadd_big(hi, lo, tot, rest + ((small + ef) + t));
}

}  // namespace ssp
