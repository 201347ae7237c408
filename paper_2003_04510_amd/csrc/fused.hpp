// Fused stage kernels of the full-RNS HE Mul.  Each kernel is one NTT pass
// (ntt.hpp) with the element-wise work of the neighbouring HE Mul step done
// in its prologue or epilogue, so that the step's operands make a single
// trip through HBM:
//
//   k_tensor_intt      tensor product (Fig. 2 region 1) + INTT "blocks" pass of d2
//   k_conv_ntt_cols    fast base conversion (mod up / mod down) + NTT "cols" pass
//   k_ntt_ip           NTT "blocks" pass + evk inner product (+ INTT "blocks"
//                      pass of the special limbs)
//   k_ntt_combine      NTT "blocks" pass + mod-down combine
//   k_lift_ntt_cols    rescale lift of the dropped limb + NTT "cols" pass
//   k_ntt_rescale      NTT "blocks" pass + rescale combine
//
// Work items are tiles (a limb x a group of columns or blocks); grids are
// padded to a multiple of 8 and items are handed out so that each XCD walks
// a contiguous item range (items that share source tiles share that XCD's
// L2).
#pragma once
#include "ntt.hpp"

namespace he {

constexpr u64 M30 = (1ull << 30) - 1;

// Item index for workgroup `bid` of a grid of `grid` (grid % 8 == 0):
// hardware places consecutive workgroups on consecutive XCDs, so XCD x
// receives items [x * grid/8, (x+1) * grid/8).
__device__ __forceinline__ u32 xcd_item(u32 bid, u32 grid) { return (bid & 7u) * (grid >> 3) + (bid >> 3); }

// ---------------------------------------------------------------- base conversion
// One conversion target: z = (sum_{s < ns} y_s * c_s) mod t, sources
// y_s = src[src_off + s], constants c_s = {c0, c1} (30-bit halves) at
// consts[c_off + 2 s].  All sources and constants are below 2^60 and
// ns <= 15, so the four partial sums of 30x30-bit products stay below 2^64.
struct ConvTarget {
  u32 src_off, ns, c_off, mi;
};

__device__ __forceinline__ u64 conv_finish(u64 sll, u64 slh, u64 shl, u64 shh, const ModInfo& m) {
  const u64 mid = slh + shl;
  const u64 cm = mid < slh ? 1 : 0;
  U128 x;
  x.lo = sll;
  x.hi = 0;
  const u64 alo = shh << 60;
  x.lo += alo;
  x.hi += (shh >> 4) + (x.lo < alo ? 1 : 0);
  const u64 blo = mid << 30;
  x.lo += blo;
  x.hi += ((mid >> 34) | (cm << 30)) + (x.lo < blo ? 1 : 0);
  return reduce128(x, m);
}

// ---------------------------------------------------------------- K1
// Tensor product + first INTT pass ("blocks") of d2.
// Items: limb i < level, block tile.  Writes d0, d1 to rl[0], rl[1], d2 (NTT
// form) to d2o, and the blocks-pass output of d2 to yp[i].  With x01 != null
// the items of limb level-1 also run the blocks pass on d0 and d1 and write
// it to x01[0], x01[1] (used to rescale without a second INTT later).
struct TensorArgs {
  const u64 *ct1, *ct2;
  u64 *rl, *d2o, *yp, *x01;
  const ModInfo* mods;
  const Tw2* itw;
  u32 level, log_n, nitems;
};

template <int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_tensor_intt(TensorArgs a) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  constexpr int FIRST = Gm::NR - 1;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= a.nitems) return;
  const int n1 = a.log_n - LOGS;
  const u32 tpl = (1u << n1) / PL::SUBS;
  const u32 i = w / tpl, pos = w % tpl;
  const u64 N = 1ull << a.log_n, tot = (u64)a.level << a.log_n;
  const ModInfo m = a.mods[i];
  const u64 blk0 = (u64)pos * PL::SUBS;
  const u64 off = ((u64)i << a.log_n) + (blk0 << LOGS);
  const int sub = PL::sub(), tt = PL::tt();
  const bool extra = a.x01 && i == a.level - 1;
  u64 d0v[Gm::R], d1v[Gm::R];
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) {
    const u64 idx = off + threadIdx.x + k * THREADS;
    const u64 b1 = a.ct1[idx], a1 = a.ct1[tot + idx], b2 = a.ct2[idx], a2 = a.ct2[tot + idx];
    d0v[k] = barrett(mul_wide(b1, b2), m);
    U128 s = mul_wide(a1, b2);
    add_to(s, mul_wide(a2, b1));
    d1v[k] = barrett(s, m);
    const u64 d2 = barrett(mul_wide(a1, a2), m);
    a.rl[idx] = d0v[k];
    a.rl[tot + idx] = d1v[k];
    a.d2o[idx] = d2;
    const int e = threadIdx.x + k * THREADS;
    lds[(e >> LOGS) * Gm::SUB + Gm::pad(e & (Gm::S - 1))] = d2;
  }
  __syncthreads();
  const Tw2* tw = a.itw + ((u64)i << a.log_n);
  const u64 base = (1ull << n1) + blk0 + sub;
  u64* tile = lds + sub * Gm::SUB;
  {
    u64* out = a.yp + off + ((u64)sub << LOGS);
    u64 x[Gm::R];
    lds_get<LOGS, LOGR, FIRST>(tile, x, tt);
    sub_transform_regs<false, LOGS, LOGR, false>(x, tile, tt, tw, base, m.q,
                                                  [&](int e, u64 v) { out[e] = csub(v, m.q); });
  }
  if (!extra) return;
#pragma unroll 1
  for (int u = 0; u < 2; ++u) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) {
      const int e = threadIdx.x + k * THREADS;
      lds[(e >> LOGS) * Gm::SUB + Gm::pad(e & (Gm::S - 1))] = u ? d1v[k] : d0v[k];
    }
    __syncthreads();
    u64* out = a.x01 + (u64)u * N + (blk0 << LOGS) + ((u64)sub << LOGS);
    u64 x[Gm::R];
    lds_get<LOGS, LOGR, FIRST>(tile, x, tt);
    sub_transform_regs<false, LOGS, LOGR, false>(x, tile, tt, tw, base, m.q,
                                                  [&](int e, u64 v) { out[e] = csub(v, m.q); });
  }
}

// ---------------------------------------------------------------- K3 / K6
// Base conversion + forward NTT "cols" pass.
// Items: (z, column tile, target o), o fastest.  Target o reads sources
// src + z*src_z + (t.src_off + s) N and writes dst + z*dst_z + o N.  When
// side != null, target side_o also stores its coefficient-form value to
// side + z*N.
struct ConvNttArgs {
  const u64* src;
  u64* dst;
  u64 src_z, dst_z;
  const ConvTarget* tg;
  const u32* consts;
  const ModInfo* mods;
  const Tw2* tw;
  u64* side;
  u32 side_o, ntarget, log_n, nitems;
};

template <int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_conv_ntt_cols(ConvNttArgs a) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, true, EPW>;
  using RF = RoundShape<LOGS, LOGR, 0>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= a.nitems) return;
  const int n2 = a.log_n - LOGS;
  const u32 tpc = (1u << n2) / PL::SUBS;
  const u32 o = w % a.ntarget, rest = w / a.ntarget;
  const u32 pos = rest % tpc, z = rest / tpc;
  const ConvTarget T = a.tg[o];
  const ModInfo m = a.mods[T.mi];
  const int sub = PL::sub(), tt = PL::tt();
  const u64 col = (u64)pos * PL::SUBS + sub;
  const u64* src = a.src + (u64)z * a.src_z + ((u64)T.src_off << a.log_n) + col;
  const u32* C = a.consts + T.c_off;
  u64 x[Gm::R];
#pragma unroll
  for (int u = 0; u < RF::NG; ++u) {
#pragma unroll
    for (int i = 0; i < RF::G; ++i) {
      const u64 e = (u64)RF::elem(tt, u, i) << n2;
      u64 sll = 0, slh = 0, shl = 0, shh = 0;
#pragma unroll
      for (int s = 0; s < 15; ++s) {
        if (s >= (int)T.ns) break;
        const u64 y = src[((u64)s << a.log_n) + e];
        const u32 y0 = (u32)(y & M30), y1 = (u32)(y >> 30);
        const u32 c0 = C[2 * s], c1 = C[2 * s + 1];
        sll += (u64)y0 * c0;
        slh += (u64)y0 * c1;
        shl += (u64)y1 * c0;
        shh += (u64)y1 * c1;
      }
      x[u * RF::G + i] = conv_finish(sll, slh, shl, shh, m);
    }
  }
  if (a.side && o == a.side_o) {
    u64* sd = a.side + ((u64)z << a.log_n) + col;
#pragma unroll
    for (int u = 0; u < RF::NG; ++u)
#pragma unroll
      for (int i = 0; i < RF::G; ++i) sd[(u64)RF::elem(tt, u, i) << n2] = x[u * RF::G + i];
  }
  u64* out = a.dst + (u64)z * a.dst_z + ((u64)o << a.log_n) + col;
  sub_transform_regs<true, LOGS, LOGR, false>(x, lds + sub * Gm::SUB, tt, a.tw + ((u64)T.mi << a.log_n), 1, m.q,
                                               [&](int e, u64 v) { out[(u64)e << n2] = ntt_canon<true>(v, m.q); });
}

// ---------------------------------------------------------------- K4
// Forward NTT "blocks" pass of every mod-up limb of target e, evk inner
// product over the digits, and (special limbs, or limb level-1 when x != 0)
// the INTT "blocks" pass of the two accumulators.
// Items: (block tile, e) with e fastest.  ks layout [2][level+K+1][N]:
// limbs < level hold ks_u in NTT form; limbs level..level+K-1 the INTT
// blocks-pass output of the special limbs; limb level+K that of limb level-1.
struct IpArgs {
  const u64* d2;      // [level][N] NTT form
  const u64* dtp;     // cols-pass output of the mod-up limbs (compact)
  const u64* evk;     // [dnum][2][L+K][N]
  u64* ks;
  const ModInfo* mods;
  const Tw2 *tw, *itw;
  const u32* emod;
  u32 dt_first[8], lo[8], cnt[8];
  u32 beta, level, K, L, log_n, nitems, extra_last;
};

template <int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_ip(IpArgs a) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  using RF = RoundShape<LOGS, LOGR, 0>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= a.nitems) return;
  const u32 ne = a.level + a.K;
  const int n1 = a.log_n - LOGS;
  const u32 e = w % ne, pos = w / ne;
  const u32 mi = a.emod[e];
  const ModInfo m = a.mods[mi];
  const u64 blk0 = (u64)pos * ((u32)PL::SUBS);
  const u64 toff = blk0 << LOGS;  // tile offset inside a limb
  const int sub = PL::sub(), tt = PL::tt();
  u64* tile = lds + sub * Gm::SUB;
  const u64 base = (1ull << n1) + blk0 + sub;
  const u64 nm = a.L + a.K;
  u64 accb[Gm::R], acca[Gm::R];
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) accb[k] = acca[k] = 0;
#pragma unroll 1
  for (u32 j = 0; j < a.beta; ++j) {
    u64 x[Gm::R];
    if (e < a.level && e >= a.lo[j] && e < a.lo[j] + a.cnt[j]) {
      const u64* p = a.d2 + ((u64)e << a.log_n) + toff;
#pragma unroll
      for (int k = 0; k < Gm::R; ++k) x[k] = p[threadIdx.x + k * THREADS];
    } else {
      const u32 o = e < a.lo[j] ? e : e - a.cnt[j];
      const u64* p = a.dtp + ((u64)(a.dt_first[j] + o) << a.log_n) + toff + ((u64)sub << LOGS);
#pragma unroll
      for (int u = 0; u < RF::NG; ++u)
#pragma unroll
        for (int i = 0; i < RF::G; ++i) x[u * RF::G + i] = p[RF::elem(tt, u, i)];
      sub_transform_regs<true, LOGS, LOGR, true>(x, tile, tt, a.tw + ((u64)mi << a.log_n), base, m.q,
                                                 [](int, u64) {});
      __syncthreads();
#pragma unroll
      for (int k = 0; k < Gm::R; ++k) {
        const int idx = threadIdx.x + k * THREADS;
        x[k] = ntt_canon<true>(lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))], m.q);
      }
      __syncthreads();
    }
    const u64* eb = a.evk + ((((u64)j * 2) * nm + mi) << a.log_n) + toff;
    const u64* ea = eb + (nm << a.log_n);
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) {
      const int idx = threadIdx.x + k * THREADS;
      accb[k] = addmod(accb[k], mulmod(x[k], eb[idx], m), m.q);
      acca[k] = addmod(acca[k], mulmod(x[k], ea[idx], m), m.q);
    }
  }
  const u64 kz = (u64)(ne + 1) << a.log_n;  // poly stride of ks
  const bool special = e >= a.level, last = a.extra_last && e == a.level - 1;
  if (!special) {
    u64* ob = a.ks + ((u64)e << a.log_n) + toff;
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) {
      const int idx = threadIdx.x + k * THREADS;
      ob[idx] = accb[k];
      ob[kz + idx] = acca[k];
    }
  }
  if (!special && !last) return;
  const u32 dst_limb = special ? e : ne;
  const Tw2* itw = a.itw + ((u64)mi << a.log_n);
#pragma unroll 1
  for (int u = 0; u < 2; ++u) {
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) {
      const int idx = threadIdx.x + k * THREADS;
      lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))] = u ? acca[k] : accb[k];
    }
    __syncthreads();
    u64 x[Gm::R];
    lds_get<LOGS, LOGR, Gm::NR - 1>(tile, x, tt);
    u64* out = a.ks + u * kz + ((u64)dst_limb << a.log_n) + toff + ((u64)sub << LOGS);
    sub_transform_regs<false, LOGS, LOGR, false>(x, tile, tt, itw, base, m.q,
                                                  [&](int ee, u64 v) { out[ee] = csub(v, m.q); });
    __syncthreads();
  }
}

// ---------------------------------------------------------------- K7
// Forward NTT "blocks" pass of z_u[i] and the mod-down combine
// rl_u[i] = rl_u[i] + (ks_u[i] - Z_u[i]) * [P^-1]_{q_i} (rl holds d_u).
// Items: (u, i, block tile), tile fastest.
struct CombineArgs {
  const u64* zp;   // [2][level][N] cols-pass output
  const u64* ks;   // [2][level+K+1][N]
  u64* rl;         // [2][level][N]
  const u64* pinv; // Shoup pairs per q_i
  const ModInfo* mods;
  const Tw2* tw;
  u32 level, K, log_n, nitems;
};

template <int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_combine(CombineArgs a) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  using RF = RoundShape<LOGS, LOGR, 0>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= a.nitems) return;
  const int n1 = a.log_n - LOGS;
  const u32 tpl = (1u << n1) / PL::SUBS;
  const u32 pos = w % tpl, ui = w / tpl, i = ui % a.level, u = ui / a.level;
  const ModInfo m = a.mods[i];
  const u64 blk0 = (u64)pos * PL::SUBS, toff = blk0 << LOGS;
  const int sub = PL::sub(), tt = PL::tt();
  u64 x[Gm::R];
  const u64* p = a.zp + ((u64)(u * a.level + i) << a.log_n) + toff + ((u64)sub << LOGS);
#pragma unroll
  for (int uu = 0; uu < RF::NG; ++uu)
#pragma unroll
    for (int ii = 0; ii < RF::G; ++ii) x[uu * RF::G + ii] = p[RF::elem(tt, uu, ii)];
  sub_transform_regs<true, LOGS, LOGR, true>(x, lds + sub * Gm::SUB, tt, a.tw + ((u64)i << a.log_n),
                                             (1ull << n1) + blk0 + sub, m.q, [](int, u64) {});
  __syncthreads();
  const u64 pw = a.pinv[2 * i], pws = a.pinv[2 * i + 1];
  const u64* ksu = a.ks + ((u64)(u * (a.level + a.K + 1) + i) << a.log_n) + toff;
  u64* rlu = a.rl + ((u64)(u * a.level + i) << a.log_n) + toff;
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) {
    const int idx = threadIdx.x + k * THREADS;
    const u64 Z = ntt_canon<true>(lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))], m.q);
    const u64 md = shoup_lazy(ksu[idx] + m.q - Z, pw, pws, m.q);
    rlu[idx] = csub(csub(rlu[idx] + md, m.q << 1), m.q);
  }
}

// ---------------------------------------------------------------- K8
// Rescale lift + forward NTT "cols" pass.  The dropped limb in coefficient
// form is either given (r != null: r[u]) or assembled as
//   r_u = x01_u + (ksx_u - zl_u) * [P^-1]_{q_l}  (mod q_l),
// i.e. INTT of rl_u[level-1] by linearity.  Then s = centered(r) mod q_i.
// Items: (u, column tile, i < level-1), i fastest.
struct LiftArgs {
  const u64 *r, *x01, *ksx, *zl;
  u64 ksx_z;        // poly stride of ksx
  u64* sp;          // [2][level-1][N]
  const u64* qlmod; // [level-1]: q_l mod q_i
  const ModInfo* mods;
  const Tw2* tw;
  u64 pw, pws;      // [P^-1]_{q_l} Shoup pair
  u32 level, log_n, nitems;
};

template <int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_lift_ntt_cols(LiftArgs a) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, true, EPW>;
  using RF = RoundShape<LOGS, LOGR, 0>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= a.nitems) return;
  const int n2 = a.log_n - LOGS;
  const u32 tpc = (1u << n2) / PL::SUBS;
  const u32 nl = a.level - 1;
  const u32 i = w % nl, rest = w / nl, pos = rest % tpc, u = rest / tpc;
  const ModInfo m = a.mods[i];
  const u64 ql = a.mods[nl].q;
  const u64 qlm = a.qlmod[i];
  const int sub = PL::sub(), tt = PL::tt();
  const u64 col = (u64)pos * PL::SUBS + sub;
  const u64 uoff = ((u64)u << a.log_n) + col;
  u64 x[Gm::R];
#pragma unroll
  for (int uu = 0; uu < RF::NG; ++uu) {
#pragma unroll
    for (int ii = 0; ii < RF::G; ++ii) {
      const u64 e = (u64)RF::elem(tt, uu, ii) << n2;
      u64 r;
      if (a.r) {
        r = a.r[uoff + e];
      } else {
        const u64 d = a.x01[uoff + e];
        const u64 k = a.ksx[(u64)u * a.ksx_z + col + e];
        const u64 zz = a.zl[uoff + e];
        r = csub(d + csub(shoup_lazy(k + ql - zz, a.pw, a.pws, ql), ql), ql);
      }
      u64 v = csub(r - mulhi(r, m.one_s) * m.q, m.q);  // r mod q_i
      if (2 * r >= ql) v = submod(v, qlm, m.q);
      x[uu * RF::G + ii] = v;
    }
  }
  u64* out = a.sp + ((u64)(u * nl + i) << a.log_n) + col;
  sub_transform_regs<true, LOGS, LOGR, false>(x, lds + sub * Gm::SUB, tt, a.tw + ((u64)i << a.log_n), 1, m.q,
                                               [&](int e, u64 v) { out[(u64)e << n2] = ntt_canon<true>(v, m.q); });
}

// ---------------------------------------------------------------- K9
// Forward NTT "blocks" pass of s_u[i] and out_u[i] = (c_u[i] - S) * [q_l^-1]_{q_i}.
// Items: (u, i < level-1, block tile), tile fastest.
struct RescaleArgs {
  const u64* sp;   // [2][level-1][N]
  const u64* c;    // [2][level][N]
  u64* out;        // [2][level-1][N]
  const u64* qlinv;
  const ModInfo* mods;
  const Tw2* tw;
  u32 level, log_n, nitems;
};

template <int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_rescale(RescaleArgs a) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  using RF = RoundShape<LOGS, LOGR, 0>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= a.nitems) return;
  const int n1 = a.log_n - LOGS;
  const u32 tpl = (1u << n1) / PL::SUBS;
  const u32 nl = a.level - 1;
  const u32 pos = w % tpl, ui = w / tpl, i = ui % nl, u = ui / nl;
  const ModInfo m = a.mods[i];
  const u64 blk0 = (u64)pos * PL::SUBS, toff = blk0 << LOGS;
  const int sub = PL::sub(), tt = PL::tt();
  u64 x[Gm::R];
  const u64* p = a.sp + ((u64)(u * nl + i) << a.log_n) + toff + ((u64)sub << LOGS);
#pragma unroll
  for (int uu = 0; uu < RF::NG; ++uu)
#pragma unroll
    for (int ii = 0; ii < RF::G; ++ii) x[uu * RF::G + ii] = p[RF::elem(tt, uu, ii)];
  sub_transform_regs<true, LOGS, LOGR, true>(x, lds + sub * Gm::SUB, tt, a.tw + ((u64)i << a.log_n),
                                             (1ull << n1) + blk0 + sub, m.q, [](int, u64) {});
  __syncthreads();
  const u64 qw = a.qlinv[2 * i], qws = a.qlinv[2 * i + 1];
  const u64* cu = a.c + ((u64)(u * a.level + i) << a.log_n) + toff;
  u64* ou = a.out + ((u64)(u * nl + i) << a.log_n) + toff;
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) {
    const int idx = threadIdx.x + k * THREADS;
    const u64 S = ntt_canon<true>(lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))], m.q);
    ou[idx] = csub(shoup_lazy(cu[idx] + m.q - S, qw, qws, m.q), m.q);
  }
}

}  // namespace he
