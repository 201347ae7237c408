// Negacyclic NTT / INTT for 64-bit limbs on gfx950.
//
// The N-point transform of Algorithm 3 (Cooley-Tukey, merged 2N-th root,
// twiddles TB_W[m + j] = psi^{bitrev(m + j)}) is split N = 2^n1 * 2^n2 into
// two passes through HBM:
//   pass "cols"  : the first n1 stages.  They couple only elements
//                  x[r + c 2^n2] with equal r, so each column r is an
//                  independent 2^n1-point transform with twiddles W[m + j].
//   pass "blocks": the last n2 stages.  They stay inside contiguous blocks
//                  of 2^n2 elements; block b is a 2^n2-point transform whose
//                  local stage m_loc uses W[m_loc (2^n1 + b) + j].
// Inside a pass a workgroup owns SUBS sub-transforms; each thread holds
// R = 2^LOGR elements of one of them in registers and runs up to LOGR stages
// per round (radix-2^LOGR).  Round 0 reads its operands straight from the
// producer (global memory or a fused prologue), the last round hands its
// results straight to the consumer; rounds in between exchange through LDS.
//
// The inverse runs the same butterfly network backwards (Gentleman-Sande
// butterflies with TB_invW, stages in reverse order): "blocks" first, then
// "cols", then the factor N^{-1} (merged with any per-limb constant).
//
// Lazy ranges (registers and LDS only): forward values live in [0, 4q)
// (Harvey's butterfly), inverse values in [0, 2q).  Every value handed to a
// consumer is canonical unless the consumer asks for the lazy value.
#pragma once
#include "modarith.hpp"

#ifndef NTT_EPW_DEFAULT
#define NTT_EPW_DEFAULT 2048
#endif
#ifndef NTT_BLOCKS_LDS_IO
#define NTT_BLOCKS_LDS_IO 1
#endif

namespace he {

// Twiddle tables are interleaved pairs {W, floor(W 2^63 / q)} per index
// (2^63-scaled Shoup companions, see shoup63_lazy).
struct Tw2 {
  u64 w, ws;
};

// Modulus constants of the butterflies.
struct NttMod {
  u64 q, q2, nq, n2q;  // q, 2q, 2^64 - q, 2^64 - 2q
  __device__ __forceinline__ explicit NttMod(u64 m) : q(m), q2(m << 1), nq(0 - m), n2q(0 - (m << 1)) {}
};

template <int LOGS, int LOGR>
struct Geo {
  static constexpr int S = 1 << LOGS;
  static constexpr int R = 1 << LOGR;
  static constexpr int T = S / R;                      // threads per sub-transform
  static constexpr int NR = (LOGS + LOGR - 1) / LOGR;  // register rounds
  static constexpr int SUB = S + (S >> 4) + 1;         // padded LDS stride (words), odd
  __device__ static __forceinline__ int pad(int e) { return e + (e >> 4); }
};

// Element indices owned by thread tt in round RD: group u, member i is
//   e = blk * span + c + i * cnt_c   with g = tt + u*T, blk = g / cnt_c, c = g % cnt_c.
template <int LOGS, int LOGR, int RD>
struct RoundShape {
  using Gm = Geo<LOGS, LOGR>;
  static constexpr int st = RD * LOGR;
  static constexpr int rr = (LOGS - st) < LOGR ? (LOGS - st) : LOGR;
  static constexpr int G = 1 << rr;
  static constexpr int NG = Gm::R / G;
  static constexpr int cnt_c = Gm::S >> (st + rr);
  static constexpr int span = Gm::S >> st;
  __device__ static __forceinline__ int elem(int tt, int u, int i) {
    const int g = tt + u * Gm::T;
    return (g / cnt_c) * span + (g % cnt_c) + i * cnt_c;
  }
  __device__ static __forceinline__ int blk(int tt, int u) { return (tt + u * Gm::T) / cnt_c; }
};

// Harvey forward butterfly: x, y in [0, 4q) -> x + w y, x - w y in [0, 4q).
__device__ __forceinline__ void bfly_fwd(u64& x, u64& y, const Tw2 t, const NttMod& M) {
  const u64 X = sub_if_ge(x, M.n2q);
  const u64 T = shoup63_lazy(y, t.w, t.ws, M.nq);
  y = (X + M.q2) - T;
  x = X + T;
}
// Gentleman-Sande inverse butterfly: x, y in [0, 2q) -> x + y, (x - y) w in [0, 2q).
__device__ __forceinline__ void bfly_inv(u64& x, u64& y, const Tw2 t, const NttMod& M) {
  const u64 X = x, Y = y;
  x = sub_if_ge(X + Y, M.n2q);
  y = shoup63_lazy((X + M.q2) - Y, t.w, t.ws, M.nq);
}

// Butterflies of round RD on the registers x[0..R) of thread tt.
template <bool FWD, int LOGS, int LOGR, int RD>
__device__ __forceinline__ void round_math(u64 (&x)[1 << LOGR], int tt, const Tw2* __restrict__ tw, u64 base,
                                           u64 q) {
  using RS = RoundShape<LOGS, LOGR, RD>;
  constexpr int G = RS::G, rr = RS::rr, st = RS::st;
  const NttMod M(q);
#pragma unroll
  for (int u = 0; u < RS::NG; ++u) {
    const u64 blk = (u64)RS::blk(tt, u);
    u64* v = x + u * G;
    if constexpr (FWD) {
#pragma unroll
      for (int k = 0; k < rr; ++k) {
        const int half = G >> (k + 1);
        const u64 mloc = 1ull << (st + k);
#pragma unroll
        for (int i = 0; i < G; ++i) {
          if (i & half) continue;
          bfly_fwd(v[i], v[i + half], tw[mloc * base + (blk << k) + (u64)(i >> (rr - k))], M);
        }
      }
    } else {
#pragma unroll
      for (int k = rr - 1; k >= 0; --k) {
        const int half = G >> (k + 1);
        const u64 mloc = 1ull << (st + k);
#pragma unroll
        for (int i = 0; i < G; ++i) {
          if (i & half) continue;
          bfly_inv(v[i], v[i + half], tw[mloc * base + (blk << k) + (u64)(i >> (rr - k))], M);
        }
      }
    }
  }
}

template <int LOGS, int LOGR, int RD>
__device__ __forceinline__ void lds_put(u64* tile, const u64 (&x)[1 << LOGR], int tt) {
  using RS = RoundShape<LOGS, LOGR, RD>;
#pragma unroll
  for (int u = 0; u < RS::NG; ++u)
#pragma unroll
    for (int i = 0; i < RS::G; ++i) tile[Geo<LOGS, LOGR>::pad(RS::elem(tt, u, i))] = x[u * RS::G + i];
}
template <int LOGS, int LOGR, int RD>
__device__ __forceinline__ void lds_get(const u64* tile, u64 (&x)[1 << LOGR], int tt) {
  using RS = RoundShape<LOGS, LOGR, RD>;
#pragma unroll
  for (int u = 0; u < RS::NG; ++u)
#pragma unroll
    for (int i = 0; i < RS::G; ++i) x[u * RS::G + i] = tile[Geo<LOGS, LOGR>::pad(RS::elem(tt, u, i))];
}

// Middle rounds 1 .. NR-2 (forward order) through LDS.
template <bool FWD, int LOGS, int LOGR, int K>
__device__ __forceinline__ void mid_rounds(u64 (&x)[1 << LOGR], u64* tile, int tt, const Tw2* __restrict__ tw,
                                           u64 base, u64 q) {
  constexpr int NR = Geo<LOGS, LOGR>::NR;
  if constexpr (K < NR - 1) {
    constexpr int RD = FWD ? K : NR - 1 - K;
    constexpr int PREV = FWD ? RD - 1 : RD + 1;
    lds_put<LOGS, LOGR, PREV>(tile, x, tt);
    __syncthreads();
    lds_get<LOGS, LOGR, RD>(tile, x, tt);
    round_math<FWD, LOGS, LOGR, RD>(x, tt, tw, base, q);
    // no barrier needed before the next lds_put: within one round every LDS
    // position belongs to exactly one thread
    mid_rounds<FWD, LOGS, LOGR, K + 1>(x, tile, tt, tw, base, q);
  }
}

// Whole sub-transform.  The first round takes its operands from load(e)
// (or, when IN_LDS, from the tile, already filled in the first round's
// element order); the last round hands element e to store(e, v) (or, when
// OUT_LDS, leaves it in the tile for a coalesced copy-out after a barrier).
// `tile` is this sub-transform's LDS area (Geo::SUB words).  A caller that
// runs several sub-transforms on the same tile back to back must place a
// barrier between them.
template <bool FWD, int LOGS, int LOGR, bool IN_LDS, bool OUT_LDS, class Load, class Store>
__device__ __forceinline__ void sub_transform(u64* tile, int tt, const Tw2* __restrict__ tw, u64 base, u64 q,
                                              Load&& load, Store&& store) {
  using Gm = Geo<LOGS, LOGR>;
  constexpr int NR = Gm::NR;
  constexpr int FIRST = FWD ? 0 : NR - 1;
  constexpr int LAST = FWD ? NR - 1 : 0;
  u64 x[Gm::R];
  if constexpr (IN_LDS) {
    lds_get<LOGS, LOGR, FIRST>(tile, x, tt);
  } else {
    using RS = RoundShape<LOGS, LOGR, FIRST>;
#pragma unroll
    for (int u = 0; u < RS::NG; ++u)
#pragma unroll
      for (int i = 0; i < RS::G; ++i) x[u * RS::G + i] = load(RS::elem(tt, u, i));
  }
  round_math<FWD, LOGS, LOGR, FIRST>(x, tt, tw, base, q);
  if constexpr (NR > 1) {
    mid_rounds<FWD, LOGS, LOGR, 1>(x, tile, tt, tw, base, q);
    constexpr int PREV = FWD ? LAST - 1 : LAST + 1;
    lds_put<LOGS, LOGR, PREV>(tile, x, tt);
    __syncthreads();
    lds_get<LOGS, LOGR, LAST>(tile, x, tt);
    round_math<FWD, LOGS, LOGR, LAST>(x, tt, tw, base, q);
  }
  if constexpr (OUT_LDS) {
    lds_put<LOGS, LOGR, LAST>(tile, x, tt);
  } else {
    using RS = RoundShape<LOGS, LOGR, LAST>;
#pragma unroll
    for (int u = 0; u < RS::NG; ++u)
#pragma unroll
      for (int i = 0; i < RS::G; ++i) store(RS::elem(tt, u, i), x[u * RS::G + i]);
  }
}

// As sub_transform, with the first round's operands already in x.
template <bool FWD, int LOGS, int LOGR, bool OUT_LDS, class Store>
__device__ __forceinline__ void sub_transform_regs(u64 (&x)[1 << LOGR], u64* tile, int tt, const Tw2* __restrict__ tw,
                                                   u64 base, u64 q, Store&& store) {
  using Gm = Geo<LOGS, LOGR>;
  constexpr int NR = Gm::NR;
  constexpr int FIRST = FWD ? 0 : NR - 1;
  constexpr int LAST = FWD ? NR - 1 : 0;
  round_math<FWD, LOGS, LOGR, FIRST>(x, tt, tw, base, q);
  if constexpr (NR > 1) {
    mid_rounds<FWD, LOGS, LOGR, 1>(x, tile, tt, tw, base, q);
    constexpr int PREV = FWD ? LAST - 1 : LAST + 1;
    lds_put<LOGS, LOGR, PREV>(tile, x, tt);
    __syncthreads();
    lds_get<LOGS, LOGR, LAST>(tile, x, tt);
    round_math<FWD, LOGS, LOGR, LAST>(x, tt, tw, base, q);
  }
  if constexpr (OUT_LDS) {
    lds_put<LOGS, LOGR, LAST>(tile, x, tt);
  } else {
    using RS = RoundShape<LOGS, LOGR, LAST>;
#pragma unroll
    for (int u = 0; u < RS::NG; ++u)
#pragma unroll
      for (int i = 0; i < RS::G; ++i) store(RS::elem(tt, u, i), x[u * RS::G + i]);
  }
}

// Canonical value of a lazy transform output.
template <bool FWD>
__device__ __forceinline__ u64 ntt_canon(u64 x, u64 q) {
  if constexpr (FWD) x = csub(x, q << 1);
  return csub(x, q);
}

// Radix per sub-transform size.
template <int LOGS>
struct Radix {
  static constexpr int LOGR = LOGS >= 9 ? 5 : (LOGS <= 6 ? 3 : 4);
};

// Workgroup shape of a pass: EPW elements (8*EPW bytes) per workgroup.
// `cols` passes put the sub index fastest (adjacent lanes read adjacent
// columns); `blocks` passes put the in-sub thread fastest.
constexpr int NTT_EPW = NTT_EPW_DEFAULT;
template <int LOGS, int EPW = NTT_EPW>
struct PassGeo {
  static constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  static constexpr int SUBS = EPW / Gm::S;
  static constexpr int THREADS = SUBS * Gm::T;
};
// threads of a pass workgroup (a plain function so it fits a macro argument)
constexpr int pass_threads(int logs, int epw) {
  return (epw >> logs) * ((1 << logs) >> (logs >= 9 ? 5 : (logs <= 6 ? 3 : 4)));
}
template <int LOGS, bool COLS, int EPW = NTT_EPW>
struct PassLayout {
  static_assert(PassGeo<LOGS, EPW>::THREADS == pass_threads(LOGS, EPW), "pass_threads");
  using Gm = typename PassGeo<LOGS, EPW>::Gm;
  static constexpr int SUBS = PassGeo<LOGS, EPW>::SUBS;
  __device__ static __forceinline__ int sub() { return COLS ? (int)threadIdx.x % SUBS : (int)threadIdx.x / Gm::T; }
  __device__ static __forceinline__ int tt() { return COLS ? (int)threadIdx.x / SUBS : (int)threadIdx.x % Gm::T; }
};

// ------------------------------------------------------------------ plain passes
// Arguments of one batched transform launch: limb l of polynomial z reads
// src + l*src_stride + z*src_zstride, writes dst likewise (in place allowed),
// works modulo mods[limb_mod[l]], and (inverse "cols" pass) multiplies by the
// Shoup pair scale[2l], scale[2l+1] instead of N^{-1} when scale != null.
struct NttArgs {
  const u64* src;
  u64* dst;
  u64 src_stride, dst_stride;
  u64 src_zstride, dst_zstride;
  const u32* limb_mod;
  const ModInfo* mods;
  const Tw2* tw;  // [nmods][N] (W or invW with companions)
  const u64* scale;
  u32 log_n;
};

template <bool FWD, int LOGS, int EPW = NTT_EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_cols(NttArgs a) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, true, EPW>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const int limb = blockIdx.y;
  const u32 mi = a.limb_mod[limb];
  const u64 q = a.mods[mi].q;
  const int n2 = a.log_n - LOGS;
  const int sub = PL::sub(), tt = PL::tt();
  const u64 col = (u64)blockIdx.x * PL::SUBS + sub;
  const auto in = gbl(a.src + (u64)limb * a.src_stride + (u64)blockIdx.z * a.src_zstride + col);
  const auto out = gbl(a.dst + (u64)limb * a.dst_stride + (u64)blockIdx.z * a.dst_zstride + col);
  u64 w = a.mods[mi].ninv, ws = a.mods[mi].ninvs;
  if (!FWD && a.scale) {
    w = a.scale[2 * (u64)limb];
    ws = a.scale[2 * (u64)limb + 1];
  }
  sub_transform<FWD, LOGS, LOGR, false, false>(
      lds + sub * Gm::SUB, tt, a.tw + ((u64)mi << a.log_n), 1, q,
      [&](int e) { return in[(u64)e << n2]; },
      [&](int e, u64 v) {
        out[(u64)e << n2] = FWD ? ntt_canon<true>(v, q) : csub(shoup_lazy(v, w, ws, q), q);
      });
}

// Blocks pass.  With LDS_IO the side whose register layout is
// thread-contiguous (forward output, inverse input) goes through LDS so that
// every global access is coalesced.
template <bool FWD, int LOGS, int EPW = NTT_EPW, bool LDS_IO = NTT_BLOCKS_LDS_IO>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_blocks(NttArgs a) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const int limb = blockIdx.y;
  const u32 mi = a.limb_mod[limb];
  const u64 q = a.mods[mi].q;
  const int n1 = a.log_n - LOGS;
  const int sub = PL::sub(), tt = PL::tt();
  const u64 blk0 = (u64)blockIdx.x * PL::SUBS;
  const u64 blk = blk0 + sub;
  const auto in0 = gbl(a.src + (u64)limb * a.src_stride + (u64)blockIdx.z * a.src_zstride + (blk0 << LOGS));
  const auto out0 = gbl(a.dst + (u64)limb * a.dst_stride + (u64)blockIdx.z * a.dst_zstride + (blk0 << LOGS));
  const auto in = in0 + ((u64)sub << LOGS);
  const auto out = out0 + ((u64)sub << LOGS);
  constexpr bool IN_LDS = LDS_IO && !FWD, OUT_LDS = LDS_IO && FWD;
  if constexpr (IN_LDS) {
    for (int idx = threadIdx.x; idx < PL::SUBS * Gm::S; idx += THREADS)
      lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))] = in0[idx];
    __syncthreads();
  }
  sub_transform<FWD, LOGS, LOGR, IN_LDS, OUT_LDS>(
      lds + sub * Gm::SUB, tt, a.tw + ((u64)mi << a.log_n), (1ull << n1) + blk, q,
      [&](int e) { return in[e]; }, [&](int e, u64 v) { out[e] = ntt_canon<FWD>(v, q); });
  if constexpr (OUT_LDS) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < PL::SUBS * Gm::S; idx += THREADS)
      out0[idx] = ntt_canon<FWD>(lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))], q);
  }
}

}  // namespace he
