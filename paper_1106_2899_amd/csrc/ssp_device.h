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

__device__ __forceinline__ uint4 draw(uint32_t purpose, uint32_t index, uint32_t gid, int64_t step, uint32_t k0,
                                      uint32_t k1)
{
    return philox(make_uint4(index | (purpose << 16), gid, (uint32_t)(uint64_t)step, (uint32_t)((uint64_t)step >> 32)),
                  k0, k1);
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

// Box-Muller normals from four words: (r1 cos t1, r1 sin t1, r2 cos t2),
// r = sqrt(-2 ln u_a), t = 2 pi u_b.
__device__ __forceinline__ v3<float> normals3_f32(uint4 w)
{
    const float u0 = u01<float>(w.x), u1 = u01<float>(w.y), u2 = u01<float>(w.z), u3 = u01<float>(w.w);
    // -2 ln u = -2 ln2 log2 u; the hardware sine/cosine take revolutions.
    const float r1 = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u0));
    const float r2 = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u2));
    return {r1 * __builtin_amdgcn_cosf(u1), r1 * __builtin_amdgcn_sinf(u1), r2 * __builtin_amdgcn_cosf(u3)};
}

__device__ __forceinline__ v3<double> normals3_f64(uint4 w)
{
    const double u0 = u01<double>(w.x), u1 = u01<double>(w.y), u2 = u01<double>(w.z), u3 = u01<double>(w.w);
    const double r1 = sqrt(-2.0 * log(u0));
    const double r2 = sqrt(-2.0 * log(u2));
    const double t1 = 2.0 * M_PI * u1;
    const double t2 = 2.0 * M_PI * u3;
    double s1, c1;
    sincos(t1, &s1, &c1);
    return {r1 * c1, r1 * s1, r2 * cos(t2)};
}

template <typename T> __device__ __forceinline__ v3<T> normals3(uint4 w);
template <> __device__ __forceinline__ v3<float> normals3<float>(uint4 w) { return normals3_f32(w); }
template <> __device__ __forceinline__ v3<double> normals3<double>(uint4 w) { return normals3_f64(w); }

// 1 - tanh(x) = 2 / (1 + e^{2x}), written to stay accurate when tanh -> 1.
__device__ __forceinline__ float one_minus_tanh(float x)
{
    const float e = __builtin_amdgcn_exp2f(2.88539008177792681472f * x);  // e^{2x}
    return 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
}
__device__ __forceinline__ double one_minus_tanh(double x) { return 2.0 / (1.0 + exp(2.0 * x)); }

// Neighbour exchange across the whole wavefront with DPP: lane i receives
// lane i+1 (from_next, wave_shl:1) or lane i-1 (from_prev, wave_shr:1); the
// lane without a source receives 0.
__device__ __forceinline__ int dpp_next_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_prev_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); }
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

}  // namespace ssp
