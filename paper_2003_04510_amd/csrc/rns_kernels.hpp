// Element-wise and base-conversion kernels of the full-RNS HE Mul.
#pragma once
#include "modarith.hpp"

namespace he {

constexpr int EW_THREADS = 256;

// ---- region 1 tensor product (Fig. 2): d0 = b1 b2, d1 = a1 b2 + a2 b1,
// d2 = a1 a2, per limb i modulo q_i, all in NTT form.
// ct: [2][level][N]; d01: [2][level][N] (d0, d1); d2: [level][N].
__global__ __launch_bounds__(EW_THREADS) void k_tensor(const u64* __restrict__ ct1,
                                                       const u64* __restrict__ ct2,
                                                       u64* __restrict__ d01, u64* __restrict__ d2,
                                                       const ModInfo* __restrict__ mods, u32 level,
                                                       u32 log_n) {
  const u64 tot = (u64)level << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  const ModInfo m = mods[idx >> log_n];
  const u64 b1 = ct1[idx], a1 = ct1[tot + idx], b2 = ct2[idx], a2 = ct2[tot + idx];
  d01[idx] = barrett(mul_wide(b1, b2), m);
  U128 s = mul_wide(a1, b2);
  add_to(s, mul_wide(a2, b1));
  d01[tot + idx] = barrett(s, m);
  d2[idx] = barrett(mul_wide(a1, a2), m);
}

// ---- fast base conversion (mod up / mod down; the Discussion section's
// "CRT right after iCRT", with the paper's delayed-modulo accumulation):
// for every target t of a job, z_t = (sum_s y_s * C[s][t]) mod t with one
// 128-bit accumulator and a single reduction per output.
struct ConvJob {
  u32 src_off;  // first source limb (relative to src base)
  u32 ns;       // number of sources
  u32 dst_off;  // first destination limb
  u32 nt;       // number of targets
  u32 c_off;    // constants C[s][t], row-major [ns][nt], offset into consts
  u32 m_off;    // target modulus indices, offset into tmods
};
constexpr int CONV_MAX_SRC = 32;

__global__ __launch_bounds__(EW_THREADS) void k_convert(const u64* __restrict__ src,
                                                        u64* __restrict__ dst,
                                                        const ConvJob* __restrict__ jobs,
                                                        const u64* __restrict__ consts,
                                                        const u32* __restrict__ tmods,
                                                        const ModInfo* __restrict__ mods, u32 log_n,
                                                        u64 src_zstride, u64 dst_zstride) {
  const ConvJob J = jobs[blockIdx.y];
  const u64 n = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  const u64 N = 1ull << log_n;
  if (n >= N) return;
  const u64* s0 = src + (u64)blockIdx.z * src_zstride + ((u64)J.src_off << log_n) + n;
  u64* d0 = dst + (u64)blockIdx.z * dst_zstride + ((u64)J.dst_off << log_n) + n;
  u64 y[CONV_MAX_SRC];
#pragma unroll
  for (int s = 0; s < CONV_MAX_SRC; ++s)
    if (s < (int)J.ns) y[s] = s0[(u64)s << log_n];
  const u64* C = consts + J.c_off;
  for (u32 t = 0; t < J.nt; ++t) {
    const ModInfo m = mods[tmods[J.m_off + t]];
    U128 acc = {0, 0};
#pragma unroll
    for (int s = 0; s < CONV_MAX_SRC; ++s)
      if (s < (int)J.ns) add_to(acc, mul_wide(y[s], C[(u64)s * J.nt + t]));
    d0[(u64)t << log_n] = reduce128(acc, m);
  }
}

// ---- evk inner product (region 2): for every limb e of the extended basis
// E_l and u in {b, a}: ks_u[e] = sum_j dt_j[e] * evk_j.u[e].
// dt_j[e] is d2[e] itself when q_e belongs to digit j, else the converted
// limb dt[dt_first[j] + (e < lo_j ? e : e - n_j)].
struct IpArgs {
  const u64* d2;      // [level][N]
  const u64* dt;      // compact ModUp output
  const u64* evk;     // [dnum][2][L+K][N]
  u64* ks;            // [2][level+K][N]
  const ModInfo* mods;
  const u32* emod;    // [level+K] modulus index of extended-basis limb e
  u32 dt_first[8];    // per digit: first compact limb
  u32 lo[8], cnt[8];  // per digit: first q index and size
  u32 beta, level, K, L, log_n;
};

__global__ __launch_bounds__(EW_THREADS) void k_inner_product(IpArgs a) {
  const u64 N = 1ull << a.log_n;
  const u64 n = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  const u32 e = blockIdx.y;
  if (n >= N) return;
  const u32 mi = a.emod[e];
  const ModInfo m = a.mods[mi];
  const u64 nm = a.L + a.K;
  U128 accb = {0, 0}, acca = {0, 0};
  for (u32 j = 0; j < a.beta; ++j) {
    u64 x;
    if (e >= a.lo[j] && e < a.lo[j] + a.cnt[j] && e < a.level) {
      x = a.d2[((u64)e << a.log_n) + n];
    } else {
      const u32 o = e < a.lo[j] ? e : e - a.cnt[j];
      x = a.dt[((u64)(a.dt_first[j] + o) << a.log_n) + n];
    }
    const u64* ev = a.evk + ((u64)j * 2 * nm << a.log_n);
    add_to(accb, mul_wide(x, ev[((u64)mi << a.log_n) + n]));
    add_to(acca, mul_wide(x, ev[((nm + mi) << a.log_n) + n]));
  }
  const u64 ne = a.level + a.K;
  a.ks[((u64)e << a.log_n) + n] = reduce128(accb, m);
  a.ks[((ne + e) << a.log_n) + n] = reduce128(acca, m);
}

// ---- ModDown combine: rl_u[i] = d_u[i] + (ks_u[i] - z_u[i]) * [P^-1]_{q_i}
// (rl holds d0, d1 on entry).  pinv: Shoup pairs per q_i.
__global__ __launch_bounds__(EW_THREADS) void k_moddown_combine(u64* __restrict__ rl,
                                                                const u64* __restrict__ ks,
                                                                const u64* __restrict__ z,
                                                                const u64* __restrict__ pinv,
                                                                const ModInfo* __restrict__ mods,
                                                                u32 level, u32 K, u32 log_n) {
  const u64 tot = (u64)level << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  const u32 i = (u32)(idx >> log_n);
  const u64 q = mods[i].q;
  const u64 w = pinv[2 * i], ws = pinv[2 * i + 1];
  const u64 ksoff = ((u64)(level + K)) << log_n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const u64 diff = ks[u * ksoff + idx] + q - z[u * tot + idx];  // (0, 2q)
    const u64 md = shoup_lazy(diff, w, ws, q);                   // [0, 2q)
    rl[u * tot + idx] = csub(csub(rl[u * tot + idx] + md, q << 1), q);
  }
}

// ---- rescale lift: s_u[i] = centered(r_u) mod q_i for i < level-1, where
// r_u in [0, ql) is the coefficient form of limb level-1 and centered(r) =
// r - ql when 2r >= ql.  qlmod[i] = ql mod q_i.
__global__ __launch_bounds__(EW_THREADS) void k_rescale_lift(const u64* __restrict__ r,
                                                             u64* __restrict__ s,
                                                             const u64* __restrict__ qlmod,
                                                             const ModInfo* __restrict__ mods,
                                                             u32 level, u64 ql, u32 log_n) {
  const u64 tot = (u64)(level - 1) << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  const u32 i = (u32)(idx >> log_n);
  const u64 n = idx & ((1ull << log_n) - 1);
  const ModInfo m = mods[i];
  const u64 N = 1ull << log_n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const u64 x = r[u * N + n];
    u64 v = csub(x - mulhi(x, m.one_s) * m.q, m.q);  // x mod q_i
    if (2 * x >= ql) v = submod(v, qlmod[i], m.q);
    s[u * tot + idx] = v;
  }
}

// ---- rescale combine: out_u[i] = (c_u[i] - s_u[i]) * [ql^-1]_{q_i}.
__global__ __launch_bounds__(EW_THREADS) void k_rescale_combine(const u64* __restrict__ c,
                                                                const u64* __restrict__ s,
                                                                u64* __restrict__ out,
                                                                const u64* __restrict__ qlinv,
                                                                const ModInfo* __restrict__ mods,
                                                                u32 level, u32 log_n) {
  const u64 tot = (u64)(level - 1) << log_n;
  const u64 idx = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
  if (idx >= tot) return;
  const u32 i = (u32)(idx >> log_n);
  const u64 q = mods[i].q;
  const u64 w = qlinv[2 * i], ws = qlinv[2 * i + 1];
  const u64 cstride = (u64)level << log_n;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const u64 diff = c[u * cstride + idx] + q - s[u * tot + idx];
    out[u * tot + idx] = csub(shoup_lazy(diff, w, ws, q), q);
  }
}

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
