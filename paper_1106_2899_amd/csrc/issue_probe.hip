// VALU issue-cost probe for gfx950 (measurement tooling, not part of the
// step path).
//
// Each probe kernel keeps eight independent registers and applies one VALU
// instruction kind to them in turn, 32 instructions per loop iteration, so
// that no instruction waits on the one before it and the loop's scalar
// control is small beside the vector work.  Launched with 8 waves on every
// SIMD (2048 workgroups of 256 threads on 256 CUs), the SIMDs are issue-bound
// and the cost of the instruction kind in SIMD cycles is
//     elapsed shader cycles / (waves per SIMD x instructions per wave).
// Each wave reads the shader clock (s_memtime) and the 100 MHz reference
// clock (s_memrealtime) before and after its loop; the host also times the
// launch with HIP events.  The instruction sequences are written as inline
// asm so that the count per iteration is exact; none of them touches memory.
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <utility>

namespace {

constexpr int kUnroll = 4;  // x 8 registers = 32 instructions per iteration

enum Op : int {
  ADD_F32, FMAC_F32, MUL_F32, FMA_F32, ADD_U32, XOR_B32, BITOP3_B32, LSHL_B32, MAD_U64_U32, MUL_HI_U32,
  MUL_LO_U32, CNDMASK_B32, DPP_MOV_B32, CVT_F32_U32, LOG_F32, EXP_F32, SQRT_F32, SIN_F32, COS_F32,
  RCP_F32, FMA_F64, ADD_F64, MUL_F64, CVT_F64_F32, CVT_F32_F64, N_OPS
};

const char* const kNames[N_OPS] = {
    "v_add_f32", "v_fmac_f32", "v_mul_f32", "v_fma_f32", "v_add_u32", "v_xor_b32", "v_bitop3_b32",
    "v_lshlrev_b32", "v_mad_u64_u32", "v_mul_hi_u32", "v_mul_lo_u32", "v_cndmask_b32", "v_mov_b32_dpp",
    "v_cvt_f32_u32", "v_log_f32", "v_exp_f32", "v_sqrt_f32", "v_sin_f32", "v_cos_f32", "v_rcp_f32",
    "v_fma_f64", "v_add_f64", "v_mul_f64", "v_cvt_f64_f32", "v_cvt_f32_f64"};

#define R8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

template <int OP>
__global__ __launch_bounds__(256) void k_probe(int iters, float* sink, uint64_t* clocks) {
  const uint32_t t = threadIdx.x + blockIdx.x * blockDim.x;
  float f[8];
  uint32_t u[8];
  double d[8];
  uint64_t w[8];
#define INIT(i)                                   \
  f[i] = 1.0f + 1e-3f * float((t + i) & 255);     \
  u[i] = t * 2654435761u + i;                     \
  d[i] = 1.0 + 1e-3 * double((t + 3 * i) & 255);  \
  w[i] = uint64_t(t) << 7 | i;
  R8(INIT)
#undef INIT
  const float fb = 1.0000001f, fc = 0.9999999f;
  const uint32_t ub = 0x9E3779B9u, uc = 0xD2511F53u;
  const double db = 1.0000000001, dc = 0.9999999999;
  const uint64_t mask = 0x5555555555555555ull;

  const uint64_t c0 = __builtin_amdgcn_s_memtime();
  const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      if constexpr (OP == ADD_F32) {
#define X(i) asm volatile("v_add_f32 %0, %0, %1" : "+v"(f[i]) : "v"(fb));
        R8(X)
#undef X
      } else if constexpr (OP == FMAC_F32) {
#define X(i) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(f[i]) : "v"(fb), "v"(fc));
        R8(X)
#undef X
      } else if constexpr (OP == MUL_F32) {
#define X(i) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(f[i]) : "v"(fb));
        R8(X)
#undef X
      } else if constexpr (OP == FMA_F32) {
#define X(i) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(f[i]) : "v"(fb), "v"(fc));
        R8(X)
#undef X
      } else if constexpr (OP == ADD_U32) {
#define X(i) asm volatile("v_add_u32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == XOR_B32) {
#define X(i) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == BITOP3_B32) {
#define X(i) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(u[i]) : "v"(ub), "v"(uc));
        R8(X)
#undef X
      } else if constexpr (OP == LSHL_B32) {
#define X(i) asm volatile("v_lshlrev_b32 %0, 1, %0" : "+v"(u[i]));
        R8(X)
#undef X
      } else if constexpr (OP == MAD_U64_U32) {
#define X(i) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(w[i]) : "v"(ub), "v"(uc) : "vcc");
        R8(X)
#undef X
      } else if constexpr (OP == MUL_HI_U32) {
#define X(i) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == MUL_LO_U32) {
#define X(i) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == CNDMASK_B32) {
#define X(i) asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(u[i]) : "v"(ub), "s"(mask));
        R8(X)
#undef X
      } else if constexpr (OP == DPP_MOV_B32) {
        // every register's last writer is 8 instructions back: no DPP read hazard
#define X(i) asm volatile("v_mov_b32_dpp %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf" : "+v"(u[i]));
        R8(X)
#undef X
      } else if constexpr (OP == CVT_F32_U32) {
#define X(i) asm volatile("v_cvt_f32_u32 %0, %1" : "=v"(f[i]) : "v"(u[i]));
        R8(X)
#undef X
      } else if constexpr (OP == LOG_F32) {
#define X(i) asm volatile("v_log_f32 %0, %0" : "+v"(f[i]));
        R8(X)
#undef X
      } else if constexpr (OP == EXP_F32) {
#define X(i) asm volatile("v_exp_f32 %0, %0" : "+v"(f[i]));
        R8(X)
#undef X
      } else if constexpr (OP == SQRT_F32) {
#define X(i) asm volatile("v_sqrt_f32 %0, %0" : "+v"(f[i]));
        R8(X)
#undef X
      } else if constexpr (OP == SIN_F32) {
#define X(i) asm volatile("v_sin_f32 %0, %0" : "+v"(f[i]));
        R8(X)
#undef X
      } else if constexpr (OP == COS_F32) {
#define X(i) asm volatile("v_cos_f32 %0, %0" : "+v"(f[i]));
        R8(X)
#undef X
      } else if constexpr (OP == RCP_F32) {
#define X(i) asm volatile("v_rcp_f32 %0, %0" : "+v"(f[i]));
        R8(X)
#undef X
      } else if constexpr (OP == FMA_F64) {
#define X(i) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(d[i]) : "v"(db), "v"(dc));
        R8(X)
#undef X
      } else if constexpr (OP == ADD_F64) {
#define X(i) asm volatile("v_add_f64 %0, %0, %1" : "+v"(d[i]) : "v"(db));
        R8(X)
#undef X
      } else if constexpr (OP == MUL_F64) {
#define X(i) asm volatile("v_mul_f64 %0, %0, %1" : "+v"(d[i]) : "v"(db));
        R8(X)
#undef X
      } else if constexpr (OP == CVT_F64_F32) {
#define X(i) asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(d[i]) : "v"(f[i]));
        R8(X)
#undef X
      } else if constexpr (OP == CVT_F32_F64) {
#define X(i) asm volatile("v_cvt_f32_f64 %0, %1" : "=v"(f[i]) : "v"(d[i]));
        R8(X)
#undef X
      }
    }
  }
  const uint64_t c1 = __builtin_amdgcn_s_memtime();
  const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
  float acc = 0.0f;
#define SUM(i) acc += f[i] + float(u[i] & 1u) + float(d[i]) + float(w[i] & 1u);
  R8(SUM)
#undef SUM
  sink[t] = acc;
  const uint32_t wave = t / 64u;
  if ((threadIdx.x & 63u) == 0u) {
    clocks[2 * wave] = c1 - c0;
    clocks[2 * wave + 1] = r1 - r0;
  }
}

template <int OP>
hipError_t launch(int blocks, int iters, float* sink, uint64_t* clocks, hipStream_t s) {
  hipLaunchKernelGGL(k_probe<OP>, dim3(blocks), dim3(256), 0, s, iters, sink, clocks);
  return hipGetLastError();
}

using LaunchFn = hipError_t (*)(int, int, float*, uint64_t*, hipStream_t);
template <int... I>
constexpr auto table(std::integer_sequence<int, I...>) {
  return std::array<LaunchFn, sizeof...(I)>{&launch<I>...};
}

}  // namespace

extern "C" {

// Number of instruction kinds and the name of kind `op` (NULL if out of range).
int ssp_probe_count() { return N_OPS; }
const char* ssp_probe_name(int op) { return (op >= 0 && op < N_OPS) ? kNames[op] : nullptr; }

// Runs probe kernel `op` with `blocks` workgroups of 256 threads and `iters`
// loop iterations (32 instructions of the kind per iteration and wave).
// Device buffers: sink [blocks*256] floats, clocks [blocks*4*2] (per wave:
// shader-clock cycles, then 100 MHz reference ticks, of its loop).  *ms gets
// the launch duration from HIP events.  Returns 0, or -1 on a bad argument
// or a HIP error.
int ssp_probe_run(int op, int blocks, int iters, float* sink, uint64_t* clocks, float* ms) {
  static const auto fns = table(std::make_integer_sequence<int, N_OPS>{});
  if (op < 0 || op >= N_OPS || blocks <= 0 || iters <= 0 || !sink || !clocks || !ms) return -1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1; }
  int rc = 0;
  if (hipEventRecord(e0, nullptr) != hipSuccess || fns[op](blocks, iters, sink, clocks, nullptr) != hipSuccess ||
      hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(ms, e0, e1) != hipSuccess)
    rc = -1;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
