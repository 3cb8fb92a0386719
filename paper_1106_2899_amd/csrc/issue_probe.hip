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
  RCP_F32, FMA_F64, ADD_F64, MUL_F64, CVT_F64_F32, CVT_F32_F64, SUB_F32, MAX_F32, MED3_F32, SUB_F32_DPP,
  MOV_B32, MOV_B64, AND_B32, OR_B32, SUB_U32, MAX_I32, ALIGNBIT_B32, LSHL_ADD_U32, ADD3_U32, PERM_B32, BFE_U32,
  LSHR_B32, BCNT_U32, MBCNT_LO, MUL_U32_U24, CNDMASK_VCC, CMP_NE_U32_VCC, CMP_LT_I32_SGPR, CMP_LT_F32_VCC,
  ADD_CO_U32, READFIRSTLANE, CMP_CNDMASK_VCC, CMP_CNDMASK_SGPR, N_OPS
};

const char* const kNames[N_OPS] = {
    "v_add_f32", "v_fmac_f32", "v_mul_f32", "v_fma_f32", "v_add_u32", "v_xor_b32", "v_bitop3_b32",
    "v_lshlrev_b32", "v_mad_u64_u32", "v_mul_hi_u32", "v_mul_lo_u32", "v_cndmask_b32", "v_mov_b32_dpp",
    "v_cvt_f32_u32", "v_log_f32", "v_exp_f32", "v_sqrt_f32", "v_sin_f32", "v_cos_f32", "v_rcp_f32",
    "v_fma_f64", "v_add_f64", "v_mul_f64", "v_cvt_f64_f32", "v_cvt_f32_f64", "v_sub_f32", "v_max_f32",
    "v_med3_f32", "v_sub_f32_dpp", "v_mov_b32", "v_mov_b64", "v_and_b32", "v_or_b32", "v_sub_u32", "v_max_i32",
    "v_alignbit_b32", "v_lshl_add_u32", "v_add3_u32", "v_perm_b32", "v_bfe_u32", "v_lshrrev_b32",
    "v_bcnt_u32_b32", "v_mbcnt_lo_u32_b32", "v_mul_u32_u24", "v_cndmask_b32 (vcc)", "v_cmp_ne_u32 (vcc)",
    "v_cmp_lt_i32_e64 (sgpr pair)", "v_cmp_lt_f32 (vcc)", "v_add_co_u32", "v_readfirstlane_b32",
    "v_cmp_lt_f32 + v_cndmask_b32 through vcc (pair)", "v_cmp_lt_f32_e64 + v_cndmask_b32_e64 through an sgpr pair (pair)"};

#define R8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

template <int OP>
__global__ __launch_bounds__(256) void k_probe(int iters, float* sink) {
  const uint32_t t = threadIdx.x + blockIdx.x * blockDim.x;
  float f[8];
  uint32_t u[8];
  double d[8];
  uint64_t w[8];
  uint32_t sg[8] = {};
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
      } else if constexpr (OP == SUB_F32) {
#define X(i) asm volatile("v_sub_f32 %0, %0, %1" : "+v"(f[i]) : "v"(fb));
        R8(X)
#undef X
      } else if constexpr (OP == MAX_F32) {
#define X(i) asm volatile("v_max_f32 %0, %0, %1" : "+v"(f[i]) : "v"(fb));
        R8(X)
#undef X
      } else if constexpr (OP == MED3_F32) {
#define X(i) asm volatile("v_med3_f32 %0, %0, %1, %2" : "+v"(f[i]) : "v"(fb), "v"(fc));
        R8(X)
#undef X
      } else if constexpr (OP == SUB_F32_DPP) {
        // every register's last writer is 8 instructions back: no DPP read hazard
#define X(i) asm volatile("v_sub_f32_dpp %0, %0, %1 row_shr:1 row_mask:0xf bank_mask:0xf" : "+v"(f[i]) : "v"(fb));
        R8(X)
#undef X
      } else if constexpr (OP == MOV_B32) {
#define X(i) asm volatile("v_mov_b32 %0, %1" : "=v"(u[i]) : "v"(u[(i + 1) & 7]));
        R8(X)
#undef X
      } else if constexpr (OP == MOV_B64) {
#define X(i) asm volatile("v_mov_b64 %0, %1" : "=v"(w[i]) : "v"(w[(i + 1) & 7]));
        R8(X)
#undef X
      } else if constexpr (OP == AND_B32) {
#define X(i) asm volatile("v_and_b32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == OR_B32) {
#define X(i) asm volatile("v_or_b32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == SUB_U32) {
#define X(i) asm volatile("v_sub_u32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == MAX_I32) {
#define X(i) asm volatile("v_max_i32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == ALIGNBIT_B32) {
#define X(i) asm volatile("v_alignbit_b32 %0, %0, %1, %2" : "+v"(u[i]) : "v"(ub), "v"(uc));
        R8(X)
#undef X
      } else if constexpr (OP == LSHL_ADD_U32) {
#define X(i) asm volatile("v_lshl_add_u32 %0, %0, 2, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == ADD3_U32) {
#define X(i) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(u[i]) : "v"(ub), "v"(uc));
        R8(X)
#undef X
      } else if constexpr (OP == PERM_B32) {
#define X(i) asm volatile("v_perm_b32 %0, %0, %1, %2" : "+v"(u[i]) : "v"(ub), "v"(uc));
        R8(X)
#undef X
      } else if constexpr (OP == BFE_U32) {
#define X(i) asm volatile("v_bfe_u32 %0, %0, 9, 23" : "+v"(u[i]));
        R8(X)
#undef X
      } else if constexpr (OP == LSHR_B32) {
#define X(i) asm volatile("v_lshrrev_b32 %0, 1, %0" : "+v"(u[i]));
        R8(X)
#undef X
      } else if constexpr (OP == BCNT_U32) {
#define X(i) asm volatile("v_bcnt_u32_b32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == MBCNT_LO) {
#define X(i) asm volatile("v_mbcnt_lo_u32_b32 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == MUL_U32_U24) {
#define X(i) asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == CNDMASK_VCC) {
#define X(i) asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(u[i]) : "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == CMP_NE_U32_VCC) {
#define X(i) asm volatile("v_cmp_ne_u32 vcc, %0, %1" : : "v"(u[i]), "v"(ub) : "vcc");
        R8(X)
#undef X
      } else if constexpr (OP == CMP_LT_I32_SGPR) {
#define X(i) asm volatile("v_cmp_lt_i32_e64 %0, %1, %2" : "=s"(w[i]) : "v"(u[i]), "v"(ub));
        R8(X)
#undef X
      } else if constexpr (OP == CMP_LT_F32_VCC) {
#define X(i) asm volatile("v_cmp_lt_f32 vcc, %0, %1" : : "v"(f[i]), "v"(fb) : "vcc");
        R8(X)
#undef X
      } else if constexpr (OP == ADD_CO_U32) {
#define X(i) asm volatile("v_add_co_u32 %0, vcc, %0, %1" : "+v"(u[i]) : "v"(ub) : "vcc");
        R8(X)
#undef X
      } else if constexpr (OP == CMP_CNDMASK_VCC) {
        // 16 compare + select pairs per iteration (32 instructions)
#define X(i)                                                                                         \
  if ((i & 1) == 0)                                                                                  \
    asm volatile("v_cmp_lt_f32 vcc, %1, %2\n\tv_cndmask_b32 %0, %0, %3, vcc" : "+v"(u[i]) : "v"(f[i]), \
                 "v"(fb), "v"(ub) : "vcc");
        R8(X) R8(X)
#undef X
      } else if constexpr (OP == CMP_CNDMASK_SGPR) {
#define X(i)                                                                                     \
  if ((i & 1) == 0) {                                                                            \
    uint64_t c;                                                                                  \
    asm volatile("v_cmp_lt_f32_e64 %1, %2, %3\n\tv_cndmask_b32_e64 %0, %0, %4, %1"              \
                 : "+v"(u[i]), "=&s"(c) : "v"(f[i]), "v"(fb), "v"(ub));                            \
  }
        R8(X) R8(X)
#undef X
      } else if constexpr (OP == READFIRSTLANE) {
#define X(i) asm volatile("v_readfirstlane_b32 %0, %1" : "=s"(sg[i]) : "v"(u[i]));
        R8(X)
#undef X
      }
    }
  }
  float acc = 0.0f;
#define SUM(i) acc += f[i] + float(u[i] & 1u) + float(d[i]) + float(w[i] & 1u) + float(sg[i] & 1u);
  R8(SUM)
#undef SUM
  sink[t] = acc;
}

template <int OP>
hipError_t launch(int blocks, int iters, float* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_probe<OP>, dim3(blocks), dim3(256), 0, s, iters, sink);
  return hipGetLastError();
}

using LaunchFn = hipError_t (*)(int, int, float*, hipStream_t);
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
// sink: device buffer of blocks*256 floats (one result per thread, so that
// the work is live).  *ms gets the launch duration from HIP events.
// Returns 0, or -1 on a bad argument or a HIP error.
int ssp_probe_run(int op, int blocks, int iters, float* sink, float* ms) {
  static const auto fns = table(std::make_integer_sequence<int, N_OPS>{});
  if (op < 0 || op >= N_OPS || blocks <= 0 || iters <= 0 || !sink || !ms) return -1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1; }
  int rc = 0;
  if (hipEventRecord(e0, nullptr) != hipSuccess || fns[op](blocks, iters, sink, nullptr) != hipSuccess ||
      hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(ms, e0, e1) != hipSuccess)
    rc = -1;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
