// Device modular arithmetic for 64-bit residues on gfx950's 32-bit integer
// ALUs.  Every 64x64 product is built from v_mad_u64_u32 / v_mul_hi_u32
// partial products.  Moduli are odd primes below 2^60.
//
//   shoup_lazy : Shoup's modular multiplication by a constant with a
//                precomputed companion (Algorithm 2), result in [0, 2q),
//                correction left to the caller (lazy range).
//   barrett    : reduction of a 128-bit value below 2^(2b+2) (b = bit length
//                of q), result canonical.
//   reduce128  : reduction of any 128-bit value with high word < 2^64 via
//                two Shoup steps (2^64 mod q and 1), result canonical.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace he {

typedef uint64_t u64;
typedef uint32_t u32;

// Read-only table access through the constant address space: with a
// uniform address this becomes a scalar load (scalar cache, lgkmcnt), so it
// never waits behind outstanding vector-memory traffic.  Only for data that
// no kernel writes while it runs (moduli, twiddles, conversion constants).
template <class T>
__device__ __forceinline__ T ldc(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized table entries");
  typedef const __attribute__((address_space(4))) uint32_t* cptr;
  const cptr src = (cptr)p;
  T r;
  uint32_t* d = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) d[i] = src[i];
  return r;
}

// HBM pointers that reach a kernel inside a struct are generic pointers to
// the compiler, which then emits flat accesses: those count against the LDS
// counter too and must be ordered against LDS accesses that might alias, so
// a load followed by an LDS store waits for the load.  Accessing HBM through
// the global address space avoids both.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> gbl(T* p) {
  return (gptr<T>)p;
}

// A value every lane of the wavefront holds, moved to a scalar register.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

struct U128 {
  u64 lo, hi;
};

__device__ __forceinline__ U128 mul_wide(u64 a, u64 b) {
  const u32 al = (u32)a, ah = (u32)(a >> 32), bl = (u32)b, bh = (u32)(b >> 32);
  const u64 p0 = (u64)al * bl, p1 = (u64)al * bh, p2 = (u64)ah * bl, p3 = (u64)ah * bh;
  const u64 mid = (p0 >> 32) + (u32)p1 + (u32)p2;
  U128 r;
  r.lo = (mid << 32) | (u32)p0;
  r.hi = p3 + (p1 >> 32) + (p2 >> 32) + (mid >> 32);
  return r;
}

__device__ __forceinline__ void add_to(U128& acc, const U128& x) {
  acc.lo += x.lo;
  acc.hi += x.hi + (acc.lo < x.lo ? 1 : 0);
}

__device__ __forceinline__ u64 mulhi(u64 a, u64 b) { return __umul64hi(a, b); }

__device__ __forceinline__ u64 csub(u64 x, u64 m) { return x >= m ? x - m : x; }

// x*w mod q in [0, 2q) for any x < 2^64; w < q, ws = floor(w 2^64 / q)
__device__ __forceinline__ u64 shoup_lazy(u64 x, u64 w, u64 ws, u64 q) {
  return x * w - mulhi(x, ws) * q;
}
__device__ __forceinline__ u64 shoup(u64 x, u64 w, u64 ws, u64 q) {
  return csub(shoup_lazy(x, w, ws, q), q);
}

// Per-modulus constants shared by all kernels.
struct ModInfo {
  u64 q;
  u64 mu;      // floor(2^(2b) / q), Barrett
  u64 r64;     // 2^64 mod q
  u64 r64s;    // Shoup companion of r64
  u64 one_s;   // floor(2^64 / q): Shoup companion of 1
  u64 ninv;    // N^{-1} mod q
  u64 ninvs;   // Shoup companion of ninv
  u32 b;       // bit length of q
  u32 arith;   // butterfly arithmetic: ARITH_AUTO (by size), ARITH_I32 (32-bit words, q < 2^30)
  double qinv; // fl(1/q)
};
constexpr u32 ARITH_AUTO = 0, ARITH_I32 = 2;

// x < 2^(2b+2): canonical x mod q.
__device__ __forceinline__ u64 barrett(U128 x, const ModInfo& m) {
  const u32 s = m.b - 1;
  const u64 x1 = (x.lo >> s) | (x.hi << (64 - s));
  const U128 p = mul_wide(x1, m.mu);
  const u32 t = m.b + 1;
  const u64 qh = (p.lo >> t) | (p.hi << (64 - t));
  u64 r = x.lo - qh * m.q;  // in [0, 7q)
  const u64 q2 = m.q << 1, q4 = m.q << 2;
  r = csub(r, q4);
  r = csub(r, q2);
  return csub(r, m.q);
}

// Any x with x.hi < 2^64: canonical x mod q.
__device__ __forceinline__ u64 reduce128(U128 x, const ModInfo& m) {
  const u64 u = shoup_lazy(x.hi, m.r64, m.r64s, m.q);    // hi * 2^64 mod q, [0, 2q)
  const u64 v = x.lo - mulhi(x.lo, m.one_s) * m.q;       // lo mod q, [0, 2q)
  u64 r = u + v;                                         // [0, 4q)
  r = csub(r, m.q << 1);
  return csub(r, m.q);
}

// Shoup multiplication with a 2^63-scaled companion ws = floor(w 2^63 / q),
// valid for x < 2^62 and q < 2^61: returns x*w mod q in [0, 2q).
// Built so every 64-bit intermediate fits: with x_hi < 2^30 and ws_hi < 2^31
// the middle partial products chain through v_mad_u64_u32 addends without
// overflow, and the remainder is formed as x*w + qhat*(2^64 - q) mod 2^64
// (additions only).  nq = 2^64 - q.
__device__ __forceinline__ u64 shoup63_lazy(u64 x, u64 w, u64 ws, u64 nq) {
  const u32 xl = (u32)x, xh = (u32)(x >> 32), wsl = (u32)ws, wsh = (u32)(ws >> 32);
  const u32 p = __umulhi(xl, wsl);
  const u64 b = (u64)xh * wsl + p;
  const u64 a = (u64)xl * wsh + b;
  const u64 h = (u64)xh * wsh + (a >> 32);
  // qhat = floor(x ws / 2^63) = (h : a_lo) >> 31
  const u32 ql = __builtin_amdgcn_alignbit((u32)h, (u32)a, 31);
  const u32 qh = __builtin_amdgcn_alignbit((u32)(h >> 32), (u32)h, 31);
  const u32 wl = (u32)w, wh = (u32)(w >> 32), nql = (u32)nq, nqh = (u32)(nq >> 32);
  u64 t = (u64)xl * wl;
  t = (u64)ql * nql + t;
  const u32 hi = (u32)(t >> 32) + xl * wh + xh * wl + ql * nqh + qh * nql;
  return ((u64)hi << 32) | (u32)t;
}

// floor(x s / 2^64) for s < 2^32 (below 2^32): the low word's product
// contributes only its high half, so two 32-bit multiplies suffice.
__device__ __forceinline__ u32 mulhi_u64_u32(u64 x, u32 s) {
  const u64 t = (u64)(u32)(x >> 32) * s + __umulhi((u32)x, s);
  return (u32)(t >> 32);
}

// x mod q in [0, 2q) for any x < 2^64 (Shoup's product by 1, companion
// one_s = floor(2^64 / q)); for q > 2^32 the companion is below 2^32.
__device__ __forceinline__ u64 mod1_lazy(u64 x, const ModInfo& m) {
  if (m.q >> 32) return x - (u64)mulhi_u64_u32(x, (u32)m.one_s) * m.q;
  return x - mulhi(x, m.one_s) * m.q;
}

// Canonical x mod q for x < 2^125 (x.hi < 2^61) and 2^32 < q < 2^61: the
// high word through the 2^63-scaled Shoup product by 2^64 mod q (whose
// companion floor(r64 2^63 / q) is r64s / 2), the low word through
// mod1_lazy.  Same value as reduce128, fewer instructions.
__device__ __forceinline__ u64 reduce125(U128 x, const ModInfo& m) {
  const u64 u = shoup63_lazy(x.hi, m.r64, m.r64s >> 1, 0 - m.q);       // [0, 2q)
  const u64 v = x.lo - (u64)mulhi_u64_u32(x.lo, (u32)m.one_s) * m.q;  // [0, 2q)
  u64 r = u + v;
  r = csub(r, m.q << 1);
  return csub(r, m.q);
}

// x - m if x >= m else x, for x, m < 2^63; negm = 2^64 - m.
__device__ __forceinline__ u64 sub_if_ge(u64 x, u64 negm) {
  const u64 t = x + negm;
  return (int64_t)t < 0 ? x : t;
}

// canonical (a*b) mod q for a, b < q
__device__ __forceinline__ u64 mulmod(u64 a, u64 b, const ModInfo& m) { return barrett(mul_wide(a, b), m); }

__device__ __forceinline__ u64 addmod(u64 a, u64 b, u64 q) { return csub(a + b, q); }
__device__ __forceinline__ u64 submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

}  // namespace he
