// Stage kernels of the full-RNS HE Mul, for one HE Mul or a batch of them.
//
// Most kernels are one NTT pass (ntt.hpp) with the element-wise work of the
// neighbouring HE Mul step done in its prologue or epilogue, so that the
// step's operands make a single trip through HBM:
//
//   k_tensor_intt      tensor product (Fig. 2 region 1) + INTT "blocks" pass of d2
//   k_list_cols        NTT / INTT "cols" pass over a limb list of a pair
//   k_list_blocks      NTT / INTT "blocks" pass over a limb list of a pair
//   k_conv             fast base conversion (mod up / mod down)
//   k_ip               evk inner product (Fig. 2 region 2)
//   k_blocks_ip        NTT "blocks" passes of the mod-up limbs + evk inner
//                      product + INTT "blocks" pass of the special limbs
//                      (the fused alternative of the three above)
//   k_lift_ntt_cols    rescale lift of the dropped limb + NTT "cols" pass
//   k_zcols_lift       the NTT "cols" pass of z and the lift in one launch
//   k_ntt_combine      NTT "blocks" passes of z and s + mod-down combine
//                      + rescale combine
//   k_ntt_rescale      NTT "blocks" pass + rescale combine (stand-alone
//                      rescale only)
//
// Work items.  A launch covers the work items of every pair of a batch: the
// items of pair p are [offs[p], offs[p+1]) (per-stage prefix sums built on
// the host); a single HE Mul is a batch of one whose descriptor travels in
// the kernel arguments.  Item counts per pair are given by stage_items();
// kernels decode items in the same order.  Grids are padded to a multiple
// of 8 and items are handed out so that each XCD walks a contiguous range.
#pragma once
#include <type_traits>

#include "ntt.hpp"

namespace he {

constexpr u64 M30 = (1ull << 30) - 1;

// Residues are stored in HBM as words of type W: uint64_t, or uint32_t for
// contexts whose primes are below 2^31 (32-bit words).  Descriptors carry
// untyped base pointers; a kernel converts a base to W before adding
// element offsets.  Arithmetic is the same for both word types: a word is
// widened on load and every stored value is canonical, so it fits W.
template <class W>
__device__ __forceinline__ gptr<W> gw(u64* p) {
  return (gptr<W>)reinterpret_cast<W*>(p);
}
template <class W>
__device__ __forceinline__ gptr<const W> gw(const u64* p) {
  return (gptr<const W>)reinterpret_cast<const W*>(p);
}

// Workgroup tiles (elements per workgroup) of the NTT passes.  Defaults:
// "cols" passes 4096 elements (16 adjacent columns at N = 2^16), "blocks"
// passes 2048; batches at N = 2^16 may select other tiles (TileCfg).
constexpr int EPW_C = 4096, EPW_B = 2048;
// fused_ip selects k_blocks_ip (mod-up NTT blocks + inner product +
// special INTT blocks in one pass, less HBM traffic) over the separate
// launches (shorter dependency chains per workgroup) for the pairs of at
// least fused_ip digits (0: none): the fused pass runs one digit per
// wavefront, so pairs of few digits leave waves idle in its NTT phase.
struct TileCfg {
  u32 epw_c = EPW_C, epw_b = EPW_B, fused_ip = 0;
  u32 logr = 0;  // log2 register radix of both NTT passes (0: the default per sub-transform size)
};
constexpr int CONV_THREADS = 256, CONV_GROUPS = 4;  // base conversion
// Coefficients per conversion thread for jobs of up to ns sources: all the
// source residues of a thread's coefficients stay in registers, so jobs of
// more than 8 sources take one coefficient per thread.
__host__ __device__ constexpr u32 conv_cpt(u32 ns) { return ns > 8 ? 1 : 2; }
constexpr int CONV_RUN = 15;  // sources whose 30x30-bit products a 64-bit sum takes without a carry
constexpr int CONV_MAXT = 32;  // targets of one conversion item (jobs of at most 4 x 32 targets)
constexpr int IP_CPT = 2, IP_THREADS = 256;                        // inner product

// Item index for workgroup `bid` of a grid of `grid` (grid % 8 == 0):
// hardware places consecutive workgroups on consecutive XCDs, so XCD x
// receives items [x * grid/8, (x+1) * grid/8).
__device__ __forceinline__ u32 xcd_item(u32 bid, u32 grid) { return (bid & 7u) * (grid >> 3) + (bid >> 3); }

// ---------------------------------------------------------------- tables
// One base-conversion target, z = (sum_{s < ns} y_s c_s) mod t, as a record
// of conv_rec_words(NSMAX) words (NSMAX: the kernel's source bound): five
// 64-bit words (t, 2^64 mod t, its Shoup companion, floor(2^64 / t), and for
// mod down q_{level-1} mod t, which the rescale's lift uses), then the
// constants c_s = {c0, c1} (30-bit halves) of sources s < NSMAX, zero past
// the job's ns sources.  A job's targets are consecutive records, so the
// address of the next target's constants depends on nothing loaded.
__host__ __device__ constexpr u32 conv_rec_words(int nsmax) { return 10 + 2 * nsmax; }
// One conversion job (a digit for mod up, the special limbs for mod down):
// targets tg[tg_off .. tg_off + nt) write limbs dst_off .. dst_off + nt.
struct ConvJobDev {
  u32 src_off, ns, dst_off, nt, tg_off, pad;
};

constexpr int MAX_DIGITS = 64;  // key-switching digits (dnum) of a context

// Per-level plan (device-resident, built once per context).
struct PlanDev {
  const ConvJobDev* mu_jobs;  // [beta]
  const u32* mu_c;            // conversion records of the mod-up targets [dt_limbs]
  const ConvJobDev* md_jobs;  // [1]
  const u32* md_c;            // ... of the mod-down targets [level]
  const u32* dt_mod;   // modulus of each mod-up limb [dt_limbs]
  const u32* dtg_limb; // mod-up limbs ordered by modulus [dt_limbs] ...
  const u32* dtg_first;// ... and where each modulus' run starts [dtg_count + 1]
  const u32* emod;     // modulus of extended-basis limb e [level + K]
  const u32* y_mod;    // INTT list d2 (+ d0, d1 of limb level-1) [level + 2]
  const u64* y_scale;  // Shoup pairs: N^-1 [(Qt_j/q_i)^-1]_{q_i}, N^-1
  const u32* s_mod;    // INTT list of the special limbs (+ limb level-1) [K + 1]
  const u64* s_scale;  // Shoup pairs: N^-1 [(P/p_k)^-1]_{p_k}, N^-1
  const u64* qlinv;    // Shoup pairs [q_{level-1}^-1]_{q_i}, i < level-1
  const u64* qlmod;    // q_{level-1} mod q_i
  u64 pinv_l, pinv_ls; // [P^-1]_{q_{level-1}} and its Shoup companion
  u32 level, beta, dt_limbs, dtg_count;
  u32 dt_first[MAX_DIGITS], lo[MAX_DIGITS], cnt[MAX_DIGITS];
};

// One HE Mul of a launch: operands, outputs, workspace, plan.
//   ct1, ct2 [2][level][N]; rl [2][level][N] (holds d0, d1 of the tensor
//   product; receives the relinearized ciphertext when wrl);
//   out [2][level-1][N] or null; r: coefficient form of the dropped limb
//   [2][N] (stand-alone rescale only, else null);
//   workspace: d2 [level], y [level+2], dt [dt_limbs], ks [2][level+K+1],
//   z [2][level], zc [2][level] (limbs of N words).  d2 and y are adjacent;
//   once the inner product has consumed them, s_u[i] of the rescale
//   (i < level-1) is written at limb u*level + i from d2 on, which stays
//   below y[level] and y[level+1] (still read by the lift).
struct PairDesc {
  const u64 *ct1, *ct2;
  u64 *rl, *out;
  const u64* r;
  u64 *d2, *y, *dt, *ks, *z, *zc;
  const PlanDev* plan;
  u32 level, rs, wrl, pad;  // rs: rescale requested; wrl: write the relinearized ciphertext to rl
};

// Per-launch constants.
struct Common {
  const ModInfo* mods;
  const Tw2 *tw, *itw;
  const u64* evk;   // [dnum][2][L+K][N]
  const u64* pinv;  // Shoup pairs [P^-1]_{q_i}
  const u32* iota;  // 0, 1, 2, ...
  u32 L, K, log_n, dnum;
  u32 bigq;         // every prime above 2^32 (the conversions' reductions then take one form)
  u32 gstride;      // words per modulus of gtw / igtw
  const double *gtw, *igtw;  // factored blocks-pass twiddles of the FP64 moduli (GenTw)
};

// Which pairs a launch covers.
// A launch may cover a contiguous range of a batch's pairs: `pairs` and
// `offs` then point at its first pair, and its items are numbered from 0
// (offs[0] is added back).
struct Batch {
  PairDesc one;            // the pair of a single HE Mul (pairs == null)
  const PairDesc* pairs;   // device array [npairs] for a batch
  const u32* offs;         // device array [npairs + 1]: item prefix of this stage
  u32 npairs, nitems;
};

__device__ __forceinline__ PairDesc resolve(const Batch& b, u32 w, u32& local) {
  if (!b.pairs) {
    local = w;
    return b.one;
  }
  w += ldc(b.offs);
  u32 lo = 0, hi = b.npairs;  // offs[lo] <= w < offs[hi]
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if (ldc(b.offs + mid) <= w) lo = mid;
    else hi = mid;
  }
  local = uniform(w - ldc(b.offs + lo));
  return ldc(b.pairs + lo);
}

// ---------------------------------------------------------------- stages
enum Stage : int {
  ST_TENSOR = 0,   // tensor + INTT blocks (d2; d0, d1 of limb level-1 when rescaling)
  ST_Y_ICOLS,      // INTT cols of y
  ST_MU_CONV,      // mod-up conversion
  ST_DT_NCOLS,     // NTT cols of the mod-up limbs
  ST_DT_NBLOCKS,   // NTT blocks of the mod-up limbs                      (separate path)
  ST_IP,           // inner product with evk, + INTT blocks of the special limbs (+ limb
                   // level-1)                                             (separate path)
  ST_KS_IBLOCKS,   // no launch: the pass runs in ST_IP or ST_BLOCKS_IP
  ST_BLOCKS_IP,    // the three above in one pass                         (fused path)
  ST_KS_ICOLS,     // INTT cols of the special limbs (+ limb level-1)
  ST_MD_CONV,      // mod-down conversion
  ST_Z_NCOLS,      // NTT cols of z, and the rescale lift + NTT cols of s (over d2 / y)
  ST_COMBINE,      // NTT blocks of z and s + combine + rescale combine
  ST_COUNT,
  // stand-alone rescale only
  ST_LIFT = ST_COUNT,  // rescale lift + NTT cols
  ST_RESCALE,          // NTT blocks + rescale combine
  // rotation only (replaces ST_TENSOR): INTT blocks of sigma_g(a), from d2 into y
  ST_Y_IBLOCKS
};

// Tiles per limb of a cols / blocks pass at ring degree 2^log_n.
__host__ __device__ constexpr u32 cols_tiles(u32 log_n, u32 epw = EPW_C) {
  return (1u << (log_n - log_n / 2)) / (epw >> (log_n / 2));
}
__host__ __device__ constexpr u32 blocks_tiles(u32 log_n, u32 epw = EPW_B) {
  return (1u << (log_n / 2)) / (epw >> (log_n - log_n / 2));
}

// The fused mod-up blocks + inner-product pass (k_blocks_ip) runs one digit
// per wavefront of an IP_WAVES-wave workgroup (so dnum <= IP_WAVES) on tiles
// of 64 / T sub-transforms per wave (T threads per sub-transform).
constexpr int IP_WAVES = 4;
__host__ __device__ constexpr u32 ipw_elems(u32 log_n) {
  return 64u * (1u << radix_log(log_n - log_n / 2));
}
__host__ __device__ constexpr u32 ipw_tiles(u32 log_n) { return (1u << log_n) / ipw_elems(log_n); }

// Work items of one pair in a stage.
inline u32 stage_items(int st, u32 log_n, u32 level, u32 K, u32 alpha, u32 beta, u32 dt_limbs, bool rs, bool wrl,
                       TileCfg tc_cfg = TileCfg{}) {
  const u32 tc = cols_tiles(log_n, tc_cfg.epw_c), tb = blocks_tiles(log_n, tc_cfg.epw_b);
  const u32 chunks_i = (1u << log_n) / (IP_THREADS * IP_CPT);
  const u32 chunks_up = (1u << log_n) / (CONV_THREADS * conv_cpt(alpha));
  const u32 chunks_down = (1u << log_n) / (CONV_THREADS * conv_cpt(K));
  const u32 ex = rs ? 1 : 0;
  const bool fused = tc_cfg.fused_ip && beta >= tc_cfg.fused_ip;
  switch (st) {
    case ST_TENSOR: return (2 * level + 2 * ex) * tb;
    case ST_Y_ICOLS: return (level + 2 * ex) * tc;
    case ST_MU_CONV: return beta * CONV_GROUPS * chunks_up;
    case ST_DT_NCOLS: return dt_limbs * tc;
    case ST_DT_NBLOCKS: return fused ? 0 : dt_limbs * tb;
    case ST_IP: return fused ? 0 : (level + K) * chunks_i;
    case ST_KS_IBLOCKS: return 0;  // in k_ip (separate path) or k_blocks_ip (fused path)
    case ST_BLOCKS_IP: return fused ? (level + K + ex) * ipw_tiles(log_n) : 0;
    case ST_KS_ICOLS: return 2 * (K + ex) * tc;
    case ST_MD_CONV: return 2 * CONV_GROUPS * chunks_down;
    case ST_Z_NCOLS: return rs ? (wrl ? 2 * level * tc + 2 * (level - 1) * tc : 2 * (level - 1) * tc) : 2 * level * tc;
    case ST_LIFT: return rs ? 2 * (level - 1) * tc : 0;
    case ST_COMBINE: return 2 * level * tb;
    case ST_RESCALE: return rs ? 2 * (level - 1) * tb : 0;
    case ST_Y_IBLOCKS: return level * tb;
  }
  return 0;
}

// ---------------------------------------------------------------- blocks-pass twiddles
// Twiddle source of the sub-transform of row block blk (of 2^(log_n - LOGS))
// in a blocks pass of modulus mi: the factored form for FP64 moduli (GenTw)
// from 512-point sub-transforms up, the table otherwise.  Up to 256 points
// the table's reads cost less than forming the twiddles: a block's share of
// the table is smaller, and limbs of one modulus that run side by side (the
// digits of mod up, the two polynomials of the combine) share it in L2.
template <class A, bool FWD, int LOGS>
__device__ __forceinline__ auto blocks_tw(const Common& c, u32 mi, u64 blk) {
  if constexpr (std::is_same<A, F64A>::value && LOGS >= 9) {
    const double* g = (FWD ? c.gtw : c.igtw) + (u64)mi * c.gstride;
    return GenTw{g, g + (1u << LOGS) + blk * LOGS};
  } else {
    return TabTw{(FWD ? c.tw : c.itw) + ((u64)mi << c.log_n), (1ull << (c.log_n - LOGS)) + blk};
  }
}

// ---------------------------------------------------------------- base conversion helpers
// sll + (slh + shl) 2^30 + shh 2^60 as a 128-bit value.
__device__ __forceinline__ U128 conv_sum(u64 sll, u64 slh, u64 shl, u64 shh) {
  typedef unsigned __int128 u128;  // add-with-carry chains instead of compares
  const u128 x = (u128)sll + ((u128)shh << 60) + (((u128)slh + shl) << 30);
  return U128{(u64)x, (u64)(x >> 64)};
}

// ---------------------------------------------------------------- tensor + INTT blocks
// Items, for r < level, in pairs over (limb r, block tile), kind fastest:
//   kind 0: d0, d1 of the tile into rl (a plain stream, no transform);
//   kind 1: d2 (NTT form) into d2 and its INTT blocks pass into y[r].
// The two items of a tile are adjacent, so they run on one XCD and the
// second reads a1, a2 from its L2; splitting the tile doubles the waves
// that hide the memory latency of a grid of about one wave per SIMD.
// Then, when rescaling, items (level + u, block tile): d_u of limb level-1
// again, its INTT blocks pass into y[level + u] (rescale by linearity).
template <class W, int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_tensor_intt(Common c, Batch b) {
  constexpr int LOGR = tile_logr(EPW, LOGS);
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  constexpr int FIRST = Gm::NR - 1;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  const int n1 = c.log_n - LOGS;
  const u32 tpl = (1u << n1) / PL::SUBS;
  const u32 npair = 2 * pd.level * tpl;
  u32 r, pos, which;  // which: 0, 1 d_u of limb level-1; 2 d2 + transform; 3 d0, d1 stream
  if (local < npair) {
    r = uniform((local >> 1) / tpl);
    pos = uniform((local >> 1) % tpl);
    which = (local & 1) ? 2 : 3;
  } else {
    r = uniform(pd.level + (local - npair) / tpl);
    pos = uniform((local - npair) % tpl);
    which = r - pd.level;
  }
  const u32 i = r < pd.level ? r : pd.level - 1;
  const u64 tot = (u64)pd.level << c.log_n;
  const ModInfo m = ldc(c.mods + i);
  const u64 blk0 = (u64)pos * PL::SUBS;
  const u64 off = ((u64)i << c.log_n) + (blk0 << LOGS);
  const int sub = PL::sub(), tt = PL::tt();
  const auto ct1 = gw<W>(pd.ct1) + off, ct2 = gw<W>(pd.ct2) + off;
  const auto put = [&](int k, u64 v) {
    const int e = threadIdx.x + k * THREADS;
    lds[(e >> LOGS) * Gm::SUB + Gm::pad(e & (Gm::S - 1))] = v;
  };
  // Operands are loaded TG elements at a time before any result is stored.
  constexpr int TG = Gm::R < 8 ? Gm::R : 8;
  if (which == 3) {
    const auto rl0 = gw<W>(pd.rl) + off, rl1 = gw<W>(pd.rl) + tot + off;
    // the products in FP64 for q < 2^50 (exact, see F64A::mulv), else on
    // the integer multipliers; both canonical
    const auto products = [&](auto f64) {
      constexpr bool F = decltype(f64)::value;
      const F64A::Mod M = F64A::mod(m.q, m.qinv);
#pragma unroll
      for (int k0 = 0; k0 < Gm::R; k0 += TG) {
        u64 b1[TG], a1[TG], b2[TG], a2[TG];
#pragma unroll
        for (int g = 0; g < TG; ++g) {
          const u64 idx = threadIdx.x + (k0 + g) * THREADS;
          // b1, b2: read by this item only (a1, a2 again by the d2 item)
          b1[g] = __builtin_nontemporal_load(&ct1[idx]); a1[g] = ct1[tot + idx];
          b2[g] = __builtin_nontemporal_load(&ct2[idx]); a2[g] = ct2[tot + idx];
        }
#pragma unroll
        for (int g = 0; g < TG; ++g) {
          const u64 idx = threadIdx.x + (k0 + g) * THREADS;
          u64 v0, v1;
          if constexpr (F) {
            const double B1 = F64A::in(b1[g], M), A1 = F64A::in(a1[g], M);
            const double B2 = F64A::in(b2[g], M), A2 = F64A::in(a2[g], M);
            v0 = F64A::to_u64(F64A::mulv(B1, B2, M), M);
            v1 = F64A::to_u64(F64A::red(F64A::mulv(A1, B2, M) + F64A::mulv(A2, B1, M), M), M);
          } else {
            U128 s1 = mul_wide(a1[g], b2[g]);
            add_to(s1, mul_wide(a2[g], b1[g]));
            v0 = barrett(mul_wide(b1[g], b2[g]), m);
            v1 = barrett(s1, m);
          }
          rl0[idx] = v0;
          rl1[idx] = v1;
        }
      }
    };
    if (f64_mod(m.q)) products(std::true_type{});
    else products(std::false_type{});
    return;
  }
  if (which == 2) {
    const auto d2 = gw<W>(pd.d2) + off;
    constexpr int TA = Gm::R < 16 ? Gm::R : 16;  // two operands: twice the loads in flight
    const auto products = [&](auto f64) {
      constexpr bool F = decltype(f64)::value;
      const F64A::Mod M = F64A::mod(m.q, m.qinv);
#pragma unroll
      for (int k0 = 0; k0 < Gm::R; k0 += TA) {
        u64 a1[TA], a2[TA];
#pragma unroll
        for (int g = 0; g < TA; ++g) {
          const u64 idx = threadIdx.x + (k0 + g) * THREADS;
          a1[g] = ct1[tot + idx]; a2[g] = ct2[tot + idx];
        }
#pragma unroll
        for (int g = 0; g < TA; ++g) {
          const u64 idx = threadIdx.x + (k0 + g) * THREADS;
          u64 v;
          if constexpr (F) {
            v = F64A::to_u64(F64A::mulv(F64A::in(a1[g], M), F64A::in(a2[g], M), M), M);
          } else {
            v = barrett(mul_wide(a1[g], a2[g]), m);
          }
          d2[idx] = v;
          put(k0 + g, v);
        }
      }
    };
    if (f64_mod(m.q)) products(std::true_type{});
    else products(std::false_type{});
  } else {  // d0 (which 0) or d1 (which 1) of limb level-1, for the rescale
    const u64 h = which == 0 ? 0 : tot;
#pragma unroll
    for (int k0 = 0; k0 < Gm::R; k0 += TG) {
      u64 x1[TG], x2[TG], y1[TG], y2[TG];
#pragma unroll
      for (int g = 0; g < TG; ++g) {
        const u64 idx = threadIdx.x + (k0 + g) * THREADS;
        x1[g] = ct1[h + idx]; y2[g] = ct2[idx];
        y1[g] = ct1[idx]; x2[g] = ct2[h + idx];
      }
#pragma unroll
      for (int g = 0; g < TG; ++g) {
        // which 0: b1 b2; which 1: a1 b2 + a2 b1
        U128 s1 = mul_wide(x1[g], y2[g]);
        if (which == 1) add_to(s1, mul_wide(x2[g], y1[g]));
        put(k0 + g, barrett(s1, m));
      }
    }
  }
  lds_barrier();
  const auto out = gw<W>(pd.y) + ((u64)r << c.log_n) + (blk0 << LOGS) + ((u64)sub << LOGS);
  u64 xi[Gm::R];
  lds_get<LOGS, LOGR, FIRST>(lds + sub * Gm::SUB, xi, tt);
  // the transform writes only tile positions this thread has just read
  // (for 8-byte values; with 4-byte values the positions differ, so every
  // thread must have read its operands first)
  with_arith<W>(m, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(m.q, m.qinv);
    typename A::V x[Gm::R];
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) x[k] = A::in(xi[k], M);
    if constexpr (sizeof(typename A::V) != 8) lds_barrier();
    sub_transform_src<A, false, LOGS, LOGR, false>(
        x, reinterpret_cast<typename A::V*>(lds) + sub * Gm::SUB, tt, blocks_tw<A, false, LOGS>(c, i, blk0 + sub), M,
        [&](int e, typename A::V v) { out[e] = A::template out<false>(v, M); });
  });
}

// ---------------------------------------------------------------- NTT passes over limb lists
struct ListView {
  const u64* src;  // base pointers (word type of the kernel) ...
  u64* dst;
  u64 so, dof;     // ... and element offsets from them
  u64 zs, zd;  // polynomial strides
  const u32* limb_mod;
  const u64* scale;  // inverse cols pass: per-limb Shoup pairs (null: N^-1)
  u32 nl, np;
};

template <int ST>
__device__ __forceinline__ ListView list_view(const Common& c, const PairDesc& pd) {
  const PlanDev* P = pd.plan;
  const u64 N = 1ull << c.log_n;
  const u32 ex = pd.rs ? 1 : 0;
  ListView v{};
  if constexpr (ST == ST_Y_ICOLS) {
    v.src = pd.y; v.dst = pd.y; v.nl = pd.level + 2 * ex; v.np = 1;
    v.limb_mod = ldc(&P->y_mod); v.scale = ldc(&P->y_scale);
  } else if constexpr (ST == ST_DT_NCOLS || ST == ST_DT_NBLOCKS) {
    v.src = pd.dt; v.dst = pd.dt; v.nl = ldc(&P->dt_limbs); v.np = 1;
    v.limb_mod = ldc(&P->dt_mod); v.scale = nullptr;
  } else if constexpr (ST == ST_KS_IBLOCKS || ST == ST_KS_ICOLS) {
    const u64 ne = pd.level + c.K;
    v.src = pd.ks; v.dst = pd.ks; v.so = v.dof = (u64)pd.level << c.log_n;
    v.zs = v.zd = (ne + 1) * N; v.nl = c.K + ex; v.np = 2;
    v.limb_mod = ldc(&P->s_mod); v.scale = ldc(&P->s_scale);
  } else if constexpr (ST == ST_Y_IBLOCKS) {
    v.src = pd.d2; v.dst = pd.y; v.nl = pd.level; v.np = 1;
    v.limb_mod = c.iota; v.scale = nullptr;
  } else {  // ST_Z_NCOLS
    v.src = pd.zc; v.dst = pd.z; v.zs = v.zd = (u64)pd.level * N; v.nl = pd.level; v.np = 2;
    v.limb_mod = c.iota; v.scale = nullptr;
  }
  return v;
}

template <class W, bool FWD, int LOGS, int EPW, int ST>
__device__ __forceinline__ void list_cols_item(const Common& c, const PairDesc& pd, u32 local, u64* lds) {
  constexpr int LOGR = tile_logr(EPW, LOGS);
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, true, EPW>;
  constexpr int FIRST = FWD ? 0 : Gm::NR - 1;
  using RF = RoundShape<LOGS, LOGR, FIRST>;
  const ListView v = list_view<ST>(c, pd);
  const int n2 = c.log_n - LOGS;
  const u32 tpc = (1u << n2) / PL::SUBS;
  const u32 pos = uniform(local % tpc), rest = local / tpc;
  const u32 z = uniform(rest % v.np), limb = uniform(rest / v.np);  // both polys of a limb adjacent
  const u32 mi = ldc(v.limb_mod + limb);
  const ModInfo mo = ldc(c.mods + mi);
  const int sub = PL::sub(), tt = PL::tt();
  const u64 col = (u64)pos * PL::SUBS + sub;
  const auto in = gw<W>(v.src) + v.so + (u64)z * v.zs + ((u64)limb << c.log_n) + col;
  const auto out = gw<W>(v.dst) + v.dof + (u64)z * v.zd + ((u64)limb << c.log_n) + col;
  u64 sw = mo.ninv, sws = mo.ninvs;
  if (!FWD && v.scale) {
    sw = ldc(v.scale + 2 * (u64)limb);
    sws = ldc(v.scale + 2 * (u64)limb + 1);
  }
  u64 xi[Gm::R];
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) xi[k] = in[(u64)RF::elem(tt, k / RF::G, k % RF::G) << n2];
  with_arith<W>(mo, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(mo.q, mo.qinv);
    const typename A::Scale sc = A::scale(sw, sws, M);
    typename A::V x[Gm::R];
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) x[k] = A::in(xi[k], M);
    sub_transform_regs<A, FWD, LOGS, LOGR, false>(
        x, reinterpret_cast<typename A::V*>(lds) + sub * Gm::SUB, tt, (FWD ? c.tw : c.itw) + ((u64)mi << c.log_n), 1,
        M, [&](int e, typename A::V val) {
          out[(u64)e << n2] = FWD ? A::template out<true>(val, M) : A::out_scaled(val, sc, M);
        });
  });
}

template <class W, bool FWD, int LOGS, int EPW, int ST>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_list_cols(Common c, Batch b) {
  __shared__ u64 lds[PassLayout<LOGS, true, EPW>::SUBS * Geo<LOGS, tile_logr(EPW, LOGS)>::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  list_cols_item<W, FWD, LOGS, EPW, ST>(c, pd, local, lds);
}

// Blocks pass; the side whose register layout is thread-contiguous
// (forward output, inverse input) goes through LDS so global accesses stay
// coalesced.
template <class W, bool FWD, int LOGS, int EPW, int ST>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_list_blocks(Common c, Batch b) {
  constexpr int LOGR = tile_logr(EPW, LOGS);
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  constexpr int FIRST = FWD ? 0 : Gm::NR - 1;
  using RF = RoundShape<LOGS, LOGR, FIRST>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  const ListView v = list_view<ST>(c, pd);
  const int n1 = c.log_n - LOGS;
  const u32 tpl = (1u << n1) / PL::SUBS;
  u32 pos, z, limb;
  if constexpr (ST == ST_DT_NBLOCKS) {
    // the mod-up limbs of one modulus (one per digit that does not contain
    // it) share their twiddles: items run tile by tile over the limbs
    // ordered by modulus, so a modulus' limbs at one tile are adjacent and
    // the later ones find the twiddles in L2
    const PlanDev* P = pd.plan;
    const u32 nl = ldc(&P->dt_limbs);
    pos = uniform(local / nl);
    limb = uniform(ldc(ldc(&P->dtg_limb) + local % nl));
    z = 0;
  } else {
    // the two polynomials of a tile adjacent: they share its twiddles
    z = uniform(local % v.np);
    const u32 rest = local / v.np;
    pos = uniform(rest % tpl);
    limb = uniform(rest / tpl);
  }
  const u32 mi = ldc(v.limb_mod + limb);
  const ModInfo mo = ldc(c.mods + mi);
  const int sub = PL::sub(), tt = PL::tt();
  const u64 blk0 = (u64)pos * PL::SUBS;
  const auto in0 = gw<W>(v.src) + v.so + (u64)z * v.zs + ((u64)limb << c.log_n) + (blk0 << LOGS);
  const auto out0 = gw<W>(v.dst) + v.dof + (u64)z * v.zd + ((u64)limb << c.log_n) + (blk0 << LOGS);
  u64 xi[Gm::R];
  if constexpr (!FWD) {
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) {
      const int idx = threadIdx.x + k * THREADS;
      lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))] = in0[idx];
    }
    lds_barrier();
    // the transform writes only tile positions this thread has just read
    lds_get<LOGS, LOGR, FIRST>(lds + sub * Gm::SUB, xi, tt);
  } else {
    const auto in = in0 + ((u64)sub << LOGS);
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) xi[k] = in[RF::elem(tt, k / RF::G, k % RF::G)];
  }
  const auto out = out0 + ((u64)sub << LOGS);
  with_arith<W>(mo, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(mo.q, mo.qinv);
    typename A::V* tl = reinterpret_cast<typename A::V*>(lds);
    typename A::V x[Gm::R];
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) x[k] = A::in(xi[k], M);
    // 4-byte values: the inverse input tile (8-byte words) is read by every
    // thread before the transform reuses it
    if constexpr (!FWD && sizeof(typename A::V) != 8) lds_barrier();
    sub_transform_src<A, FWD, LOGS, LOGR, FWD>(x, tl + sub * Gm::SUB, tt, blocks_tw<A, FWD, LOGS>(c, mi, blk0 + sub), M,
                                               [&](int e, typename A::V val) { out[e] = A::template out<FWD>(val, M); });
    if constexpr (FWD) {
      lds_barrier();
#pragma unroll
      for (int k = 0; k < Gm::R; ++k) {
        const int idx = threadIdx.x + k * THREADS;
        out0[idx] = A::template out<true>(tl[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))], M);
      }
    }
  });
}

// ---------------------------------------------------------------- base conversion
// Fast base conversion (the matrix form of the paper's iCRT, Algorithm 6,
// with its delayed modulo): a thread owns conv_cpt(NSMAX) consecutive
// coefficients, loads each source residue once (split into 30-bit halves),
// then loops over a group of targets, accumulating four 64-bit sums of
// 30x30-bit products (no carries for up to 15 sources, runs of 15 folded
// into 128 bits beyond that) and reducing once.
// Mod up: sources y, outputs dt (jobs = digits).  Mod down: sources the
// special limbs of ks (coefficient form), outputs zc, one job per polynomial.
// Mod-down constants carry P^-1 ([P/p_k]_t [P^-1]_t), so zc holds z P^-1.
// Items (job or polynomial, coefficient chunk, target group), group fastest.
// NSMAX bounds the number of sources (the digit size for mod up, K for mod
// down): all NSMAX source loads are issued unconditionally (index clamped to
// the job's ns, constants of unused sources zero), so each thread waits for
// its loads once instead of once per source.
template <class W, bool MD, int NSMAX, bool BIGQ>
__global__ __launch_bounds__(CONV_THREADS) void k_conv(Common c, Batch b) {
  constexpr int CPT = conv_cpt(NSMAX);
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  const PlanDev* P = pd.plan;
  const u32 nch = (1u << c.log_n) / (CONV_THREADS * CPT);
  // the target groups of a chunk are adjacent items (same XCD, same time),
  // so their repeated source loads hit L2
  const u32 grp = uniform(local % CONV_GROUPS), rest = local / CONV_GROUPS;
  const u32 chunk = uniform(rest % nch), jz = uniform(rest / nch);
  const ConvJobDev J = ldc((MD ? ldc(&P->md_jobs) : ldc(&P->mu_jobs)) + (MD ? 0 : jz));
  constexpr u32 RW = conv_rec_words(NSMAX);
  const u32* recs = (MD ? ldc(&P->md_c) : ldc(&P->mu_c)) + (u64)J.tg_off * RW;
  const u64 N = 1ull << c.log_n;
  const u64 ne1 = pd.level + c.K + 1;
  const auto src = MD ? gw<W>(pd.ks) + (u64)jz * ne1 * N : gw<W>(pd.y);
  const auto dst = MD ? gw<W>(pd.zc) + (u64)jz * pd.level * N : gw<W>(pd.dt);
  // merged rescale (mod down, rescaling, relinearized value not an output):
  // targets q_0 .. q_{l-2} receive z'_t + [r]_t, see below
  const bool merged = MD && pd.rs && !pd.wrl;
  const u32 nt = merged ? J.nt - 1 : J.nt;
  const u32 per = (nt + CONV_GROUPS - 1) / CONV_GROUPS;
  const u32 t0 = uniform(grp * per), t1 = uniform(min(nt, t0 + per));
  if (t0 >= t1) return;
  const u64 n0 = ((u64)chunk * CONV_THREADS + threadIdx.x) * CPT;
  const auto s0 = src + ((u64)J.src_off << c.log_n) + n0;
  u32 y0[NSMAX][CPT], y1[NSMAX][CPT];
#pragma unroll
  for (int s = 0; s < NSMAX; ++s) {
    const u32 sc = min((u32)s, J.ns - 1);
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const u64 y = s0[((u64)sc << c.log_n) + k];
      y0[s][k] = (u32)(y & M30);
      y1[s][k] = (u32)(y >> 30);
    }
  }
  // The item's target records (see conv_rec_words); slot i holds target
  // t0 + i, slot t1 - t0 the dropped limb's target (merged rescale).  Mod
  // down stages them in LDS right behind its source loads, so per target the
  // constants come from LDS, whose loads complete in order and can run
  // ahead of the arithmetic, rather than from scalar loads, which the
  // compiler re-issues next to each use and waits on target by target
  // (measured: 23.2 -> 21.1 us at n16_L24).  Mod up, and mod down from 12
  // sources on, read them with scalar loads: there the constants' VGPRs
  // would cost a wave per SIMD.
  constexpr bool LREC = MD && NSMAX <= 8;
  __shared__ u64 lrec64[LREC ? (CONV_MAXT + 1) * RW / 2 : 2];
  u32* const lrec = reinterpret_cast<u32*>(lrec64);
  if constexpr (LREC) {
    const auto g = gbl(recs);
    const u32 nw = (t1 - t0) * RW;
    for (u32 i = threadIdx.x; i < nw; i += CONV_THREADS) lrec[i] = g[(u64)t0 * RW + i];
    if (merged)
      for (u32 i = threadIdx.x; i < RW; i += CONV_THREADS) lrec[nw + i] = g[(u64)(pd.level - 1) * RW + i];
    lds_barrier();
  }
  // the record of slot `slot` in the table (the last slot, when merged, is
  // target level-1)
  const auto rec_of = [&](u32 slot) -> u64 { return merged && slot == t1 - t0 ? pd.level - 1 : t0 + slot; };
  const auto rec32 = [&](u32 slot, u32 i) -> u32 {
    if constexpr (LREC) return lrec[slot * RW + i];
    else return ldc(recs + rec_of(slot) * RW + i);
  };
  const auto rec64 = [&](u32 slot, u32 i) -> u64 {
    if constexpr (LREC) return lrec64[slot * (RW / 2) + i];
    else return ldc(reinterpret_cast<const u64*>(recs + rec_of(slot) * RW) + i);
  };
  // sum_s y_s c_s mod t for the target in record slot `slot`, canonical.
  // The 64-bit partial sums take up to 15 sources without a carry; longer
  // jobs fold each run of 15 into a 128-bit total before the one reduction.
  const auto modulus = [&](u32 slot) {
    ModInfo m{};
    m.q = rec64(slot, 0);
    m.r64 = rec64(slot, 1);
    m.r64s = rec64(slot, 2);
    m.one_s = rec64(slot, 3);
    return m;
  };
  const auto convert = [&](u32 slot, u64 (&v)[CPT]) {
    const ModInfo m = modulus(slot);
    U128 tot[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) tot[k] = U128{0, 0};
#pragma unroll
    for (int s0 = 0; s0 < NSMAX; s0 += CONV_RUN) {
      u64 sll[CPT], slh[CPT], shl[CPT], shh[CPT];
#pragma unroll
      for (int k = 0; k < CPT; ++k) sll[k] = slh[k] = shl[k] = shh[k] = 0;
#pragma unroll
      for (int s = s0; s < s0 + CONV_RUN && s < NSMAX; ++s) {
        const u32 c0 = rec32(slot, 10 + 2 * s), c1 = rec32(slot, 11 + 2 * s);
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          sll[k] += (u64)y0[s][k] * c0;
          slh[k] += (u64)y0[s][k] * c1;
          shl[k] += (u64)y1[s][k] * c0;
          shh[k] += (u64)y1[s][k] * c1;
        }
      }
#pragma unroll
      for (int k = 0; k < CPT; ++k) add_to(tot[k], conv_sum(sll[k], slh[k], shl[k], shh[k]));
    }
    // one form per launch (BIGQ: every modulus above 2^32), so the body of
    // a target has no branch and the next record's loads stay ahead of it
#pragma unroll
    for (int k = 0; k < CPT; ++k) v[k] = BIGQ ? reduce125(tot[k], m) : reduce128(tot[k], m);  // tot < 2^125
  };
  // The rescale's dropped limb in coefficient form, by linearity: with the
  // mod-down constants carrying P^-1 (z' = z P^-1),
  //   r_u = INTT(d_u[l-1]) + INTT(ks_u[l-1]) [P^-1]_{q_{l-1}} - z'_u[l-1]
  // where INTT(d_u[l-1]) = y[level + u] and INTT(ks_u[l-1]) = ks_u[level + K].
  const auto dropped = [&](const u64 (&zl)[CPT], u64 (&r)[CPT]) {
    const u64 ql = ldc(&c.mods[pd.level - 1].q);
    const u64 pw = ldc(&P->pinv_l), pws = ldc(&P->pinv_ls);
    const auto yy = gw<W>(pd.y) + ((u64)(pd.level + jz) << c.log_n) + n0;
    const auto kk = src + ((u64)(pd.level + c.K) << c.log_n) + n0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const u64 a = csub(yy[k] + csub(shoup_lazy(kk[k], pw, pws, ql), ql), ql);
      r[k] = submod(a, zl[k], ql);
    }
  };
  if (merged) {
    // Every group forms r (one more target), then each output is
    // z'_t + [r]_t with r lifted centred; the NTT of that sum is
    // NTT(z) P^-1 + NTT(s), so one transform serves mod down and rescale.
    u64 r[CPT];
    {
      u64 zl[CPT];
      convert(t1 - t0, zl);
      dropped(zl, r);
    }
    const u64 ql = ldc(&c.mods[pd.level - 1].q);
    for (u32 t = t0; t < t1; ++t) {
      u64 v[CPT];
      convert(t - t0, v);
      const ModInfo m = modulus(t - t0);
      const u64 qm = rec64(t - t0, 4);
      const auto o = dst + ((u64)t << c.log_n) + n0;
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        const u64 rq = BIGQ ? (u64)mulhi_u64_u32(r[k], (u32)m.one_s) : mulhi(r[k], m.one_s);
        u64 s = csub(r[k] - rq * m.q, m.q);               // r mod q_t
        if (2 * r[k] >= ql) s = submod(s, qm, m.q);  // centred
        o[k] = csub(v[k] + s, m.q);
      }
    }
    return;
  }
  for (u32 t = t0; t < t1; ++t) {
    u64 v[CPT];
    convert(t - t0, v);
    const auto o = dst + ((u64)(J.dst_off + t) << c.log_n) + n0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) o[k] = v[k];
    if constexpr (MD) {
      // rescaling with the relinearized value as an output: r_u replaces
      // y[level + u] for the lift
      if (pd.rs && t == pd.level - 1) {
        u64 r[CPT];
        dropped(v, r);
        const auto yy = gw<W>(pd.y) + ((u64)(pd.level + jz) << c.log_n) + n0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) yy[k] = r[k];
      }
    }
  }
}

// Smallest source bound bucket covering ns (ns <= 15).
inline int conv_bucket(u32 ns) {
  return ns <= 4 ? 4 : ns <= 8 ? 8 : ns <= 12 ? 12 : ns <= 15 ? 15 : ns <= 24 ? 24 : 32;
}

// ---------------------------------------------------------------- inner product
// ks_u[e] = sum_j dt_j[e] * evk_j.u[e] for every limb e of the extended basis;
// dt_j[e] = d2[e] when q_e is in digit j, else the NTT-form mod-up limb.
// The special limbs leave in coefficient-bound form: an item's chunk holds
// whole sub-transforms of the inverse NTT blocks pass (2^LOGS points), so
// their sums go through that pass here, by way of LDS, and the special
// limbs never make the round trip through HBM in NTT form.  When
// rescaling, ks_u[level-1] is written in NTT form and, inverse-transformed
// the same way, into slot level+K.  Both leave the inverse cols pass.
// Items in eight blocks of coefficient chunks (one per XCD for a single
// pair), limb-major inside a block: every XCD takes its share of the
// special limbs' transforms, and the workgroups in flight on it read a few
// limbs' adjacent chunks.  KEY_NT: the key is read by one HE Mul (a single
// pair), so its loads bypass the caches.
template <class W, bool KEY_NT, int LOGS>
__global__ __launch_bounds__(IP_THREADS) void k_ip(Common c, Batch b) {
  // radix-4 rounds (radix 8 from 512 points): the transforms of an item
  // then occupy its four waves, and the kernel stays at 64 VGPRs, 8 waves
  // per SIMD (the default radix 8 takes 77: 6 waves per SIMD)
  constexpr int LOGR = LOGS >= 9 ? 3 : 2;
  using Gm = Geo<LOGS, LOGR>;
  constexpr int EI = IP_THREADS * IP_CPT;  // coefficients per item
  constexpr int SUBS = EI / Gm::S;         // sub-transforms per polynomial and item
  static_assert(SUBS >= 1 && EI % Gm::S == 0, "an item holds whole blocks-pass sub-transforms");
  static_assert(64 % Gm::T == 0, "a sub-transform's threads lie in one wavefront");
  __shared__ u64 lds[2 * SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  const PlanDev* P = pd.plan;
  const u32 nel = pd.level + c.K;
  // items in 8 chunk blocks (one per XCD when the item count is a multiple
  // of 8), limb-major inside a block: each XCD takes its share of the
  // special limbs' transforms, and a limb's chunks stay adjacent
  const u32 nch = (1u << c.log_n) / (IP_THREADS * IP_CPT), cpb = nch / 8, blk = nel * cpb;
  const u32 rem = local % blk;
  const u32 e = uniform(rem / cpb), chunk = uniform((local / blk) * cpb + rem % cpb);
  const u64 n0 = ((u64)chunk * IP_THREADS + threadIdx.x) * IP_CPT;
  const u32 mi = ldc(ldc(&P->emod) + e);
  const ModInfo m = ldc(c.mods + mi);
  const u64 nm = c.L + c.K;
  const u32 beta = ldc(&P->beta);
  U128 accb[IP_CPT], acca[IP_CPT];
#pragma unroll
  for (int k = 0; k < IP_CPT; ++k) accb[k] = acca[k] = U128{0, 0};
  // Digits are taken JG at a time; all their loads are issued before any
  // accumulation (indices of digits past beta are clamped, their terms zeroed).
  constexpr int JG = 3;
  for (u32 j0 = 0; j0 < beta; j0 += JG) {
    u64 xv[JG][IP_CPT], bv[JG][IP_CPT], av[JG][IP_CPT];
#pragma unroll
    for (int jj = 0; jj < JG; ++jj) {
      const u32 j = min(j0 + jj, beta - 1);
      const u32 lo = ldc(&P->lo[j]), cnt = ldc(&P->cnt[j]);
      gptr<const W> x;
      if (e < pd.level && e >= lo && e < lo + cnt) {
        x = gw<W>((const u64*)pd.d2) + ((u64)e << c.log_n);
      } else {
        const u32 o = e < lo ? e : e - cnt;
        x = gw<W>((const u64*)pd.dt) + ((u64)(ldc(&P->dt_first[j]) + o) << c.log_n);
      }
      const auto eb = gw<W>(c.evk) + ((((u64)j * 2) * nm + mi) << c.log_n);
      const auto ea = eb + (nm << c.log_n);
#pragma unroll
      for (int k = 0; k < IP_CPT; ++k) {
        // the mod-up limbs (last use) stay out of the caches, and so does
        // the key when one HE Mul reads it (the pairs of a batch share it):
        // the caches then keep the intermediates of the stages that follow
        xv[jj][k] = __builtin_nontemporal_load(&x[n0 + k]);
        if constexpr (KEY_NT) {
          bv[jj][k] = __builtin_nontemporal_load(&eb[n0 + k]);
          av[jj][k] = __builtin_nontemporal_load(&ea[n0 + k]);
        } else {
          bv[jj][k] = eb[n0 + k];
          av[jj][k] = ea[n0 + k];
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < JG; ++jj) {
      const bool use = j0 + jj < beta;  // a select, not a branch, keeps the loads above
#pragma unroll
      for (int k = 0; k < IP_CPT; ++k) {
        const u64 xm = use ? xv[jj][k] : 0;
        add_to(accb[k], mul_wide(xm, bv[jj][k]));
        add_to(acca[k], mul_wide(xm, av[jj][k]));
      }
    }
  }
  const u64 kz = (u64)(pd.level + c.K + 1) << c.log_n;
  const bool last = pd.rs && e == pd.level - 1;
  const bool coef = e >= pd.level || last;  // goes through the inverse blocks pass
  u64 vb[IP_CPT], va[IP_CPT];
#pragma unroll
  for (int k = 0; k < IP_CPT; ++k) {
    // beta <= 4: the sums stay below 4 q^2 < 2^(2b+2), Barrett's range
    vb[k] = beta <= 4 ? barrett(accb[k], m) : reduce128(accb[k], m);
    va[k] = beta <= 4 ? barrett(acca[k], m) : reduce128(acca[k], m);
  }
  if (e < pd.level) {
    const auto ob = gw<W>(pd.ks) + ((u64)e << c.log_n) + n0;
#pragma unroll
    for (int k = 0; k < IP_CPT; ++k) {
      ob[k] = vb[k];
      ob[kz + k] = va[k];
    }
  }
  if (!coef) return;
  // inverse blocks pass: tile z * SUBS + s holds sub-transform s of
  // polynomial z (b, a); the transform's threads are whole sub-transforms
  // of one wavefront each, the rest of the workgroup is done
  with_arith<W>(m, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(m.q, m.qinv);
    typename A::V* const tl = reinterpret_cast<typename A::V*>(lds);
#pragma unroll
    for (int k = 0; k < IP_CPT; ++k) {
      const int idx = threadIdx.x * IP_CPT + k;
      const int q = (idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1));
      tl[q] = A::in(vb[k], M);
      tl[SUBS * Gm::SUB + q] = A::in(va[k], M);
    }
    lds_barrier();
    if (threadIdx.x >= 2 * SUBS * Gm::T) return;
    const int g = threadIdx.x / Gm::T, tt = threadIdx.x % Gm::T;
    const int z = g / SUBS, sub = g % SUBS;
    typename A::V x[Gm::R];
    lds_get<LOGS, LOGR, Gm::NR - 1>(tl + g * Gm::SUB, x, tt);
    const u64 blk = (u64)chunk * SUBS + sub;  // the sub-transform's block in the limb
    const u64 slot = last ? pd.level + c.K : e;
    const auto out = gw<W>(pd.ks) + (z ? kz : 0) + (slot << c.log_n) + (blk << LOGS);
    sub_transform_src<A, false, LOGS, LOGR, false, true>(
        x, tl + g * Gm::SUB, tt, blocks_tw<A, false, LOGS>(c, mi, blk), M,
        [&](int e2, typename A::V v) { out[e2] = A::template out<false>(v, M); });
  });
}

// ---------------------------------------------------------------- mod-up NTT blocks + inner product
// One workgroup per (limb e of the extended basis, tile of IPW_BLOCKS
// blocks); wave j of its IP_WAVES waves owns digit j: it runs the NTT
// blocks pass of the mod-up limb of digit j with target e on the tile (or
// takes d2[e] itself, already in NTT form, when e lies in digit j) into its
// own LDS tile, synchronizing with wave-level LDS ordering only.  After one
// workgroup barrier every thread sums the inner-product terms
//   ks_u[e] = sum_j dt_j[e] * evk_j.u[e]   (u = b, a)
// for its elements, so the NTT-form mod-up limbs never return to HBM and
// the digits of one target share their twiddles.  q limbs e < level are
// written in NTT form; special limbs, and when rescaling limb level-1 once
// more (into slot level+K), go through the inverse NTT blocks pass (waves
// 0 and 1, one polynomial each), leaving them the inverse cols pass.
// Items (e, tile), tile fastest; e < level + K (+1).

template <class W, int LOGS>
__global__ __launch_bounds__(64 * IP_WAVES) void k_blocks_ip(Common c, Batch b) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  constexpr int SUBS = 64 / Gm::T;      // sub-transforms per wave
  constexpr int EW = SUBS * Gm::S;       // elements per tile
  constexpr int TILE = SUBS * Gm::SUB;   // LDS words per wave tile
  constexpr int THREADS = 64 * IP_WAVES;
  constexpr int PER = EW / THREADS;      // elements per thread in the sum
  using RF = RoundShape<LOGS, LOGR, 0>;
  constexpr int IFIRST = Gm::NR - 1;
  static_assert(EW % THREADS == 0, "tile");
  __shared__ u64 lds[IP_WAVES * TILE];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  const PlanDev* P = pd.plan;
  const int n1 = c.log_n - LOGS;
  const u32 tpl = (1u << n1) / SUBS;
  const u32 pos = uniform(local % tpl), el = uniform(local / tpl);
  const bool copy = el == pd.level + c.K;  // ks_u[level-1] again, inverse-transformed into slot level+K
  const u32 e = copy ? pd.level - 1 : el;
  const bool coef = copy || e >= pd.level;  // leaves after the inverse blocks pass
  const u32 mi = ldc(ldc(&P->emod) + e);
  const ModInfo m = ldc(c.mods + mi);
  const u64 nm = c.L + c.K;
  const u32 beta = ldc(&P->beta);
  const u64 blk0 = (u64)pos * SUBS, toff = blk0 << LOGS;
  const u32 wave = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int sub = lane / Gm::T, tt = lane % Gm::T;
  const u64 base = (1ull << n1) + blk0 + sub;
  const auto lpos = [](int idx) { return (idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1)); };
  const u64 kz = (u64)(pd.level + c.K + 1) << c.log_n;
  with_arith<W>(m, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(m.q, m.qinv);
    typename A::V* const tiles = reinterpret_cast<typename A::V*>(lds);
    typename A::V* const mine = tiles + wave * TILE;
    // phase 1: wave j puts digit j's term of target e, NTT form, into its tile
    if (wave < beta) {
      const u32 j = wave;
      const u32 lo = ldc(&P->lo[j]), cnt = ldc(&P->cnt[j]);
      if (e < pd.level && e >= lo && e < lo + cnt) {
        const auto x = gw<W>(pd.d2) + ((u64)e << c.log_n) + toff;
#pragma unroll
        for (int k = 0; k < EW / 64; ++k) {
          const int idx = lane + k * 64;
          mine[lpos(idx)] = A::in(x[idx], M);
        }
      } else {
        const u32 o = e < lo ? e : e - cnt;
        const auto src = gw<W>(pd.dt) + ((u64)(ldc(&P->dt_first[j]) + o) << c.log_n) + toff + ((u64)sub << LOGS);
        typename A::V x[Gm::R];
#pragma unroll
        for (int k = 0; k < Gm::R; ++k) x[k] = A::in(src[RF::elem(tt, k / RF::G, k % RF::G)], M);
        sub_transform_src<A, true, LOGS, LOGR, true, true>(x, mine + sub * Gm::SUB, tt,
                                                           blocks_tw<A, true, LOGS>(c, mi, base - (1ull << n1)), M,
                                                           [](int, typename A::V) {});
      }
    }
    // phase 2 operands: the evk values of this thread's elements for every
    // digit, issued before the barrier so they arrive while waves wait
    // (digits past beta clamp to the last one; their terms are skipped)
    u64 vb[IP_WAVES][PER], va[IP_WAVES][PER];
#pragma unroll
    for (int j = 0; j < IP_WAVES; ++j) {
      const u32 jc = min((u32)j, beta - 1);
      const auto eb = gw<W>(c.evk) + ((((u64)jc * 2) * nm + mi) << c.log_n) + toff;
      const auto ea = eb + (nm << c.log_n);
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = threadIdx.x + k * THREADS;
        vb[j][k] = eb[idx];
        va[j][k] = ea[idx];
      }
    }
    lds_barrier();
    // phase 2: the sums, PER elements per thread
    u64 sb[PER], sa[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) sb[k] = sa[k] = 0;
#pragma unroll
    for (int j = 0; j < IP_WAVES; ++j) {
      if ((u32)j >= beta) break;
      const typename A::V* const tj = tiles + j * TILE;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = threadIdx.x + k * THREADS;
        const u64 xv = A::template out<true>(tj[lpos(idx)], M);
        u64 pb, pa;
        if constexpr (std::is_same<A, F64A>::value) {
          const double X = F64A::in(xv, M);
          pb = F64A::to_u64(F64A::mulv(X, F64A::in(vb[j][k], M), M), M);
          pa = F64A::to_u64(F64A::mulv(X, F64A::in(va[j][k], M), M), M);
        } else {
          pb = barrett(mul_wide(xv, vb[j][k]), m);
          pa = barrett(mul_wide(xv, va[j][k]), m);
        }
        sb[k] = addmod(sb[k], pb, m.q);
        sa[k] = addmod(sa[k], pa, m.q);
      }
    }
    if (!coef) {
      const auto ob = gw<W>(pd.ks) + ((u64)e << c.log_n) + toff;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = threadIdx.x + k * THREADS;
        ob[idx] = sb[k];
        ob[kz + idx] = sa[k];
      }
      return;
    }
    // phase 3: inverse blocks pass of the sums; tile 0 <- b, tile 1 <- a
    lds_barrier();  // every tile read above
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int q = lpos(threadIdx.x + k * THREADS);
      tiles[q] = A::in(sb[k], M);
      tiles[TILE + q] = A::in(sa[k], M);
    }
    lds_barrier();
    if (wave < 2) {
      typename A::V x[Gm::R];
      lds_get<LOGS, LOGR, IFIRST>(mine + sub * Gm::SUB, x, tt);
      const u64 slot = copy ? pd.level + c.K : e;
      const auto out = gw<W>(pd.ks) + (wave ? kz : 0) + (slot << c.log_n) + toff + ((u64)sub << LOGS);
      sub_transform_src<A, false, LOGS, LOGR, false, true>(
          x, mine + sub * Gm::SUB, tt, blocks_tw<A, false, LOGS>(c, mi, base - (1ull << n1)), M,
          [&](int e2, typename A::V v) { out[e2] = A::template out<false>(v, M); });
    }
  });
}

// ---------------------------------------------------------------- NTT blocks + combine + rescale
// v_u[i] = d_u[i] + ks_u[i] [P^-1]_{q_i} - NTT(z'_u[i])  (rl holds d_u,
// z' = z P^-1), the relinearized ciphertext, written to rl when requested
// (wrl).  When rescaling, for i < level-1 also
//   out_u[i] = (v_u[i] - NTT(s_u[i])) * [q_{l-1}^-1]_{q_i}:
// with rl an output, s_u (over d2) takes a second transform here; without
// it, the mod-down conversion already added s to z', so z holds the NTT
// input of z' + s and out_u[i] = v_u[i] * [q_{l-1}^-1]_{q_i}.  v never
// makes a trip through HBM unless it is an output.
// Items (i, u, block tile), tile fastest.
template <class W, int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_combine(Common c, Batch b) {
  constexpr int LOGR = tile_logr(EPW, LOGS);
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  using RF = RoundShape<LOGS, LOGR, 0>;
  // two tiles: NTT(z) stays in the first while s (when transformed here)
  // goes through the second, and the epilogue reads both from LDS
  __shared__ u64 lds[2 * PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  const int n1 = c.log_n - LOGS;
  const u32 tpl = (1u << n1) / PL::SUBS;
  const u32 pos = uniform(local % tpl), ui = local / tpl;
  const u32 u = uniform(ui & 1), i = uniform(ui >> 1);  // b and a of limb i adjacent (shared twiddles)
  const bool resc = pd.rs && i + 1 < pd.level;
  if (!resc && !pd.wrl) return;  // the dropped limb with no relinearized output
  const PlanDev* P = pd.plan;
  const ModInfo m = ldc(c.mods + i);
  const u64 blk0 = (u64)pos * PL::SUBS, toff = blk0 << LOGS;
  const int sub = PL::sub(), tt = PL::tt();
  const u64 limb_off = ((u64)(u * pd.level + i) << c.log_n) + toff;
  u64 xi[Gm::R];
  const auto zp = gw<W>(pd.z) + limb_off + ((u64)sub << LOGS);
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) xi[k] = zp[RF::elem(tt, k / RF::G, k % RF::G)];
  const u64 pw = ldc(c.pinv + 2 * i), pws = ldc(c.pinv + 2 * i + 1);
  const auto ksu = gw<W>(pd.ks) + ((u64)(u * (pd.level + c.K + 1) + i) << c.log_n) + toff;
  const auto rlu = gw<W>(pd.rl) + limb_off;
  const auto sp = gw<W>(pd.d2) + limb_off + ((u64)sub << LOGS);
  const auto ou = gw<W>(pd.out) + ((u64)(u * (pd.level - 1) + i) << c.log_n) + toff;
  u64 qw = 0, qws = 0;
  if (resc) {
    const u64* ql = ldc(&P->qlinv);
    qw = ldc(ql + 2 * i);
    qws = ldc(ql + 2 * i + 1);
  }
  const u64 base = (1ull << n1) + blk0 + sub;
  with_arith<W>(m, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(m.q, m.qinv);
    typename A::V* tl = reinterpret_cast<typename A::V*>(lds);
    typename A::V x[Gm::R];
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) x[k] = A::in(xi[k], M);
    const auto tws = blocks_tw<A, true, LOGS>(c, i, base - (1ull << n1));
    sub_transform_src<A, true, LOGS, LOGR, true>(x, tl + sub * Gm::SUB, tt, tws, M, [](int, typename A::V) {});
    typename A::V* const ts = tl + PL::SUBS * Gm::SUB;  // NTT(s)
    const bool two = resc && pd.wrl;  // s not merged into z
    if (two) {
#pragma unroll
      for (int k = 0; k < Gm::R; ++k) x[k] = A::in(sp[RF::elem(tt, k / RF::G, k % RF::G)], M);
      sub_transform_src<A, true, LOGS, LOGR, true>(x, ts + sub * Gm::SUB, tt, tws, M, [](int, typename A::V) {});
    }
    lds_barrier();
    // NTT(z) (and NTT(s)) of element idx, in the coalesced epilogue order
    const auto lz = [&](int idx) { return (idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1)); };
    constexpr int TG = Gm::R < 8 ? Gm::R : 8;  // loads in flight before the stores
#pragma unroll
    for (int k0 = 0; k0 < Gm::R; k0 += TG) {
      u64 kv[TG], dv[TG];
#pragma unroll
      for (int g = 0; g < TG; ++g) {
        const int idx = threadIdx.x + (k0 + g) * THREADS;
        // last reads of ks and d; the output is not read again by the HE Mul
        kv[g] = __builtin_nontemporal_load(&ksu[idx]);
        dv[g] = __builtin_nontemporal_load(&rlu[idx]);
      }
#pragma unroll
      for (int g = 0; g < TG; ++g) {
        const int idx = threadIdx.x + (k0 + g) * THREADS;
        const u64 md = shoup_lazy(kv[g], pw, pws, m.q);  // [0, 2q)
        const u64 v = csub(csub(dv[g] + md + m.q - A::template out<true>(tl[lz(idx)], M), m.q << 1), m.q);
        if (pd.wrl) rlu[idx] = v;
        if (resc) {
          const u64 S = two ? A::template out<true>(ts[lz(idx)], M) : 0;
          __builtin_nontemporal_store((W)csub(shoup_lazy(v + m.q - S, qw, qws, m.q), m.q), &ou[idx]);
        }
      }
    }
  });
}

// ---------------------------------------------------------------- rescale lift + NTT cols
// The dropped limb in coefficient form r_u is pd.r (stand-alone rescale) or
// y[level + u] (assembled by the mod-down conversion, see k_conv).  Then
// s = centered(r) mod q_i.
// Items (u, column tile, i < level-1), i fastest.
template <class W, int LOGS, int EPW>
__device__ __forceinline__ void lift_item(const Common& c, const PairDesc& pd, u32 local, u64* lds) {
  constexpr int LOGR = tile_logr(EPW, LOGS);
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, true, EPW>;
  using RF = RoundShape<LOGS, LOGR, 0>;
  const PlanDev* P = pd.plan;
  const int n2 = c.log_n - LOGS;
  const u32 tpc = (1u << n2) / PL::SUBS;
  const u32 nl = pd.level - 1;
  const u32 i = uniform(local % nl), rest = local / nl;
  const u32 pos = uniform(rest % tpc), u = uniform(rest / tpc);
  const ModInfo m = ldc(c.mods + i);
  const u64 ql = ldc(&c.mods[nl].q);
  const u64 qlm = ldc(ldc(&P->qlmod) + i);
  const int sub = PL::sub(), tt = PL::tt();
  const u64 N = 1ull << c.log_n;
  const u64 col = (u64)pos * PL::SUBS + sub;
  // r_u: pd.r (stand-alone rescale) or y[level + u], where the mod-down
  // conversion left it
  const auto rr = pd.r ? gw<W>(pd.r) + (u64)u * N + col : gw<W>((const u64*)pd.y) + ((u64)(pd.level + u) << c.log_n) + col;
  u64 x[Gm::R];
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) x[k] = rr[(u64)RF::elem(tt, k / RF::G, k % RF::G) << n2];
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) {
    const u64 r = x[k];
    u64 v = csub(mod1_lazy(r, m), m.q);  // r mod q_i
    if (2 * r >= ql) v = submod(v, qlm, m.q);
    x[k] = v;
  }
  const auto out = gw<W>(pd.d2) + ((u64)(u * pd.level + i) << c.log_n) + col;
  with_arith<W>(m, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(m.q, m.qinv);
    typename A::V xa[Gm::R];
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) xa[k] = A::in(x[k], M);
    sub_transform_regs<A, true, LOGS, LOGR, false>(
        xa, reinterpret_cast<typename A::V*>(lds) + sub * Gm::SUB, tt, c.tw + ((u64)i << c.log_n), 1, M,
        [&](int e, typename A::V v) { out[(u64)e << n2] = A::template out<true>(v, M); });
  });
}

template <class W, int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_lift_ntt_cols(Common c, Batch b) {
  __shared__ u64 lds[PassLayout<LOGS, true, EPW>::SUBS * Geo<LOGS, tile_logr(EPW, LOGS)>::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  lift_item<W, LOGS, EPW>(c, pd, local, lds);
}

// NTT cols pass of z' (mod-down) and, when rescaling with rl an output, the
// lift + NTT cols pass of s, in one launch: items [0, 2 level tiles) are
// z's, the rest s's.  The two touch disjoint buffers (z cols: zc -> z; lift:
// y -> s over d2).  Rescaling without rl as an output, s is already in z'
// and only limbs i < level-1 are transformed.
template <class W, int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_zcols_lift(Common c, Batch b) {
  __shared__ u64 lds[PassLayout<LOGS, true, EPW>::SUBS * Geo<LOGS, tile_logr(EPW, LOGS)>::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  const u32 nz = uniform(2 * (pd.rs && !pd.wrl ? pd.level - 1 : pd.level) * cols_tiles(c.log_n, tile_elems(EPW)));
  if (local < nz) list_cols_item<W, true, LOGS, EPW, ST_Z_NCOLS>(c, pd, local, lds);
  else lift_item<W, LOGS, EPW>(c, pd, local - nz, lds);
}

// ---------------------------------------------------------------- rotation: automorphism
// sigma_g (X -> X^g, g odd) of a ciphertext in NTT form, as a permutation of
// the evaluation points: entry k holds the value at psi^(2 brv(k) + 1), so
// sigma_g(a)[k] = a[k'] with 2 brv(k') + 1 = (2 brv(k) + 1) g mod 2N.
// Writes the triple key switching expects: rl = (sigma_g(b), 0), d2 = sigma_g(a).
// One thread per (limb, coefficient) of [level][N].
static __global__ __launch_bounds__(256) void k_automorphism(const u64* ct, u64* rl, u64* d2, u64 g, u32 level,
                                                      u32 log_n) {
  const u64 N = 1ull << log_n, tot = (u64)level * N;
  const u64 t = (u64)blockIdx.x * 256 + threadIdx.x;
  if (t >= tot) return;
  const u64 k = t & (N - 1), base = t - k;
  const u64 j = __brev((u32)k) >> (32 - log_n);
  const u64 e = ((2 * j + 1) * g) & (2 * N - 1);
  const u64 ks = __brev((u32)((e - 1) >> 1)) >> (32 - log_n);
  const auto in = gbl(ct);
  const auto r = gbl(rl), d = gbl(d2);
  r[t] = in[base + ks];
  r[tot + t] = 0;
  d[t] = in[tot + base + ks];
}

// ---------------------------------------------------------------- NTT blocks + rescale combine
// out_u[i] = (rl_u[i] - NTT(s_u[i])) * [q_{l-1}^-1]_{q_i}; s lives over d2.
// Items (i < level-1, u, block tile), tile fastest.
template <class W, int LOGS, int EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_rescale(Common c, Batch b) {
  constexpr int LOGR = tile_logr(EPW, LOGS);
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  using RF = RoundShape<LOGS, LOGR, 0>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const u32 w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= b.nitems) return;
  u32 local;
  const PairDesc pd = resolve(b, uniform(w), local);
  const PlanDev* P = pd.plan;
  const int n1 = c.log_n - LOGS;
  const u32 tpl = (1u << n1) / PL::SUBS;
  const u32 nl = pd.level - 1;
  const u32 pos = uniform(local % tpl), ui = local / tpl;
  const u32 u = uniform(ui & 1), i = uniform(ui >> 1);  // b and a of limb i adjacent (shared twiddles)
  const ModInfo m = ldc(c.mods + i);
  const u64 blk0 = (u64)pos * PL::SUBS, toff = blk0 << LOGS;
  const int sub = PL::sub(), tt = PL::tt();
  u64 xi[Gm::R];
  const auto p = gw<W>(pd.d2) + ((u64)(u * pd.level + i) << c.log_n) + toff + ((u64)sub << LOGS);
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) xi[k] = p[RF::elem(tt, k / RF::G, k % RF::G)];
  const u64* ql = ldc(&P->qlinv);
  const u64 qw = ldc(ql + 2 * i), qws = ldc(ql + 2 * i + 1);
  const auto cu = gw<W>(pd.rl) + ((u64)(u * pd.level + i) << c.log_n) + toff;
  const auto ou = gw<W>(pd.out) + ((u64)(u * nl + i) << c.log_n) + toff;
  with_arith<W>(m, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(m.q, m.qinv);
    typename A::V* tl = reinterpret_cast<typename A::V*>(lds);
    typename A::V x[Gm::R];
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) x[k] = A::in(xi[k], M);
    sub_transform_src<A, true, LOGS, LOGR, true>(x, tl + sub * Gm::SUB, tt, blocks_tw<A, true, LOGS>(c, i, blk0 + sub),
                                                 M, [](int, typename A::V) {});
    lds_barrier();
    constexpr int TG = Gm::R < 8 ? Gm::R : 8;  // loads in flight before the stores
#pragma unroll
    for (int k0 = 0; k0 < Gm::R; k0 += TG) {
      u64 cv[TG];
#pragma unroll
      for (int g = 0; g < TG; ++g) cv[g] = cu[threadIdx.x + (k0 + g) * THREADS];
#pragma unroll
      for (int g = 0; g < TG; ++g) {
        const int idx = threadIdx.x + (k0 + g) * THREADS;
        const u64 S = A::template out<true>(tl[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))], M);
        ou[idx] = csub(shoup_lazy(cv[g] + m.q - S, qw, qws, m.q), m.q);
      }
    }
  });
}

}  // namespace he
