// Element-wise kernels of key generation, encryption and decryption.
#pragma once
#include "modarith.hpp"

namespace he {

constexpr int EW_THREADS = 256;

// ---- key generation / encryption / decryption helpers ----
// out[l][n] = v[n] mod (modulus limb_mod[l]) for a signed small vector v.
__global__ __launch_bounds__(EW_THREADS) void k_small_to_limbs(const int64_t* __restrict__ v,
                                                               u64* __restrict__ out,
                                                               const u32* __restrict__ limb_mod,
                                                               const ModInfo* __restrict__ mods,
                                                               u32 nlimbs, u32 log_n) {
  const u64 tot = (u64)nlimbs << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  const u64 q = mods[limb_mod[idx >> log_n]].q;
  const int64_t x = v[idx & ((1ull << log_n) - 1)];
  const u64 ax = x < 0 ? (u64)(-x) : (u64)x;
  u64 r = ax % q;
  if (x < 0 && r) r = q - r;
  out[idx] = r;
}

// out[l][n] = (a[l][n] * s[l][n] + e[l][n] + add[l][n]) mod q (add may be null)
__global__ __launch_bounds__(EW_THREADS) void k_mul_add(const u64* __restrict__ a,
                                                        const u64* __restrict__ s,
                                                        const u64* __restrict__ e,
                                                        u64* __restrict__ out,
                                                        const u32* __restrict__ limb_mod,
                                                        const ModInfo* __restrict__ mods,
                                                        u32 nlimbs, u32 log_n) {
  const u64 tot = (u64)nlimbs << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  const ModInfo m = mods[limb_mod[idx >> log_n]];
  out[idx] = addmod(barrett(mul_wide(a[idx], s[idx]), m), e[idx], m.q);
}

// evk digit j: b[i] = a[i]*s[i] + e[i] + (q_i in digit j ? [P]_{q_i} s2[i] : 0)
__global__ __launch_bounds__(EW_THREADS) void k_evk_b(const u64* __restrict__ a,
                                                      const u64* __restrict__ s,
                                                      const u64* __restrict__ s2,
                                                      const u64* __restrict__ e,
                                                      u64* __restrict__ b,
                                                      const u64* __restrict__ pmod,
                                                      const ModInfo* __restrict__ mods,
                                                      u32 nlimbs, u32 dlo, u32 dhi, u32 log_n) {
  const u64 tot = (u64)nlimbs << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  const u32 i = (u32)(idx >> log_n);
  const ModInfo m = mods[i];
  u64 v = addmod(barrett(mul_wide(a[idx], s[idx]), m), e[idx], m.q);
  if (i >= dlo && i < dhi) v = addmod(v, barrett(mul_wide(pmod[i], s2[idx]), m), m.q);
  b[idx] = v;
}

// out[l][n] = x[l][n] * y[l][n] mod q  (s^2 for the evk)
__global__ __launch_bounds__(EW_THREADS) void k_mul(const u64* __restrict__ x,
                                                    const u64* __restrict__ y, u64* __restrict__ out,
                                                    const u32* __restrict__ limb_mod,
                                                    const ModInfo* __restrict__ mods, u32 nlimbs,
                                                    u32 log_n) {
  const u64 tot = (u64)nlimbs << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  out[idx] = barrett(mul_wide(x[idx], y[idx]), mods[limb_mod[idx >> log_n]]);
}

// decryption: out[i] = b[i] - a[i] * s[i] mod q_i
__global__ __launch_bounds__(EW_THREADS) void k_dec(const u64* __restrict__ ct,
                                                    const u64* __restrict__ s, u64* __restrict__ out,
                                                    const ModInfo* __restrict__ mods, u32 level,
                                                    u32 log_n) {
  const u64 tot = (u64)level << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  const ModInfo m = mods[idx >> log_n];
  out[idx] = submod(ct[idx], barrett(mul_wide(ct[tot + idx], s[idx]), m), m.q);
}

// out[l][n] = (x[l][n] + y[l][n]) mod q
__global__ __launch_bounds__(EW_THREADS) void k_add(const u64* __restrict__ x,
                                                    const u64* __restrict__ y, u64* __restrict__ out,
                                                    const u32* __restrict__ limb_mod,
                                                    const ModInfo* __restrict__ mods, u32 nlimbs,
                                                    u32 log_n) {
  const u64 tot = (u64)nlimbs << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  out[idx] = addmod(x[idx], y[idx], mods[limb_mod[idx >> log_n]].q);
}

}  // namespace he
