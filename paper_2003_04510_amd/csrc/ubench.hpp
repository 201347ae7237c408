// Issue-rate microbenchmarks of the vector ALU instructions the HE Mul is
// made of: they give the measured peaks the per-stage VALU fractions are
// taken against.  Each thread runs CHAINS independent dependency chains of
// one instruction kind (enough independent work to hide the instruction
// latency), the grid holds several waves per SIMD, and the result of every
// chain is stored so that nothing is eliminated.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace he {
namespace ub {

constexpr int CHAINS = 8;
constexpr int THREADS = 256;

enum Kind { MAD_U64_U32 = 0, MUL_HI_U32 = 1, MUL_LO_U32 = 2, FMA_F64 = 3, ADD_U32 = 4, KINDS = 5 };

// v_mad_u64_u32: acc = lo32(acc) * m + acc
__global__ __launch_bounds__(THREADS) void k_peak_mad(uint32_t iters, uint32_t m, uint64_t* sink) {
  uint64_t a[CHAINS];
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) a[i] = threadIdx.x + 977u * i + blockIdx.x;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) a[i] = (uint64_t)(uint32_t)a[i] * m + a[i];
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) s ^= a[i];
  sink[blockIdx.x * THREADS + threadIdx.x] = s;
}

// v_mul_hi_u32: x = mulhi(x, m)
__global__ __launch_bounds__(THREADS) void k_peak_mulhi(uint32_t iters, uint32_t m, uint64_t* sink) {
  uint32_t a[CHAINS];
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) a[i] = ~(threadIdx.x + 977u * i + blockIdx.x);
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) a[i] = __umulhi(a[i], m);
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) s ^= a[i];
  sink[blockIdx.x * THREADS + threadIdx.x] = s;
}

// v_mul_lo_u32: x = x * m
__global__ __launch_bounds__(THREADS) void k_peak_mullo(uint32_t iters, uint32_t m, uint64_t* sink) {
  uint32_t a[CHAINS];
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) a[i] = threadIdx.x + 977u * i + blockIdx.x;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) a[i] = a[i] * m;
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) s ^= a[i];
  sink[blockIdx.x * THREADS + threadIdx.x] = s;
}

// v_fma_f64: d = d * x + y
__global__ __launch_bounds__(THREADS) void k_peak_fma64(uint32_t iters, uint32_t m, uint64_t* sink) {
  double a[CHAINS];
  const double x = 1.0 + 1.0 / (double)(m | 1), y = 1e-3;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) a[i] = (double)(threadIdx.x + i);
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) a[i] = __builtin_fma(a[i], x, y);
  }
  double s = 0;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) s += a[i];
  sink[blockIdx.x * THREADS + threadIdx.x] = (uint64_t)__double_as_longlong(s);
}

// v_lshl_add_u32 (one full-rate 32-bit integer instruction): x = (x << 1) + m
__global__ __launch_bounds__(THREADS) void k_peak_add(uint32_t iters, uint32_t m, uint64_t* sink) {
  uint32_t a[CHAINS];
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) a[i] = threadIdx.x + 977u * i + blockIdx.x;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) a[i] = (a[i] << 1) + m;
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) s ^= a[i];
  sink[blockIdx.x * THREADS + threadIdx.x] = s;
}

}  // namespace ub
}  // namespace he
