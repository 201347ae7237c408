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
  const u64* in = a.src + (u64)limb * a.src_stride + (u64)blockIdx.z * a.src_zstride + col;
  u64* out = a.dst + (u64)limb * a.dst_stride + (u64)blockIdx.z * a.dst_zstride + col;
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
  const u64* in0 = a.src + (u64)limb * a.src_stride + (u64)blockIdx.z * a.src_zstride + (blk0 << LOGS);
  u64* out0 = a.dst + (u64)limb * a.dst_stride + (u64)blockIdx.z * a.dst_zstride + (blk0 << LOGS);
  const u64* in = in0 + ((u64)sub << LOGS);
  u64* out = out0 + ((u64)sub << LOGS);
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

// ------------------------------------------------------------------ persistent passes
// A grid of G workgroups walks the tiles t = blockIdx.x, +G, ...; while one
// tile is transformed, the next tile's operands are already in flight
// (register double buffer), so HBM traffic overlaps the butterflies.
// Tile t of a launch over nl limbs x np polynomials: z = t / (nl * TPL),
// limb = (t / TPL) % nl, position = t % TPL (TPL tiles per limb).
struct TileId {
  u32 z, limb, pos;
};
__device__ __forceinline__ u32 uniform(u32 v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ TileId tile_id(u32 t, u32 nl, u32 tpl) {
  TileId r;
  r.pos = uniform(t % tpl);
  const u32 lz = t / tpl;
  r.limb = uniform(lz % nl);
  r.z = uniform(lz / nl);
  return r;
}

template <bool FWD, int LOGS, int EPW = NTT_EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_cols_p(NttArgs a, u32 nl, u32 ntiles) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, true, EPW>;
  constexpr int FIRST = FWD ? 0 : Gm::NR - 1;
  using RF = RoundShape<LOGS, LOGR, FIRST>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const int n2 = a.log_n - LOGS;
  const u32 tpl = (1u << n2) / PL::SUBS;
  const int sub = PL::sub(), tt = PL::tt();
  u32 t = blockIdx.x;
  if (t >= ntiles) return;
  u64 nx[Gm::R];
  auto fetch = [&](u32 tile) {
    const TileId id = tile_id(tile, nl, tpl);
    const u64* in = a.src + (u64)id.limb * a.src_stride + (u64)id.z * a.src_zstride + (u64)id.pos * PL::SUBS + sub;
#pragma unroll
    for (int u = 0; u < RF::NG; ++u)
#pragma unroll
      for (int i = 0; i < RF::G; ++i) nx[u * RF::G + i] = in[(u64)RF::elem(tt, u, i) << n2];
  };
  fetch(t);
  for (; t < ntiles; t += gridDim.x) {
    u64 x[Gm::R];
#pragma unroll
    for (int i = 0; i < Gm::R; ++i) x[i] = nx[i];
    if (t + gridDim.x < ntiles) fetch(t + gridDim.x);
    const TileId id = tile_id(t, nl, tpl);
    const u32 mi = a.limb_mod[id.limb];
    const u64 q = a.mods[mi].q;
    u64* out = a.dst + (u64)id.limb * a.dst_stride + (u64)id.z * a.dst_zstride + (u64)id.pos * PL::SUBS + sub;
    u64 w = a.mods[mi].ninv, ws = a.mods[mi].ninvs;
    if (!FWD && a.scale) {
      w = a.scale[2 * (u64)id.limb];
      ws = a.scale[2 * (u64)id.limb + 1];
    }
    sub_transform_regs<FWD, LOGS, LOGR, false>(x, lds + sub * Gm::SUB, tt, a.tw + ((u64)mi << a.log_n), 1, q,
        [&](int e, u64 v) {
          out[(u64)e << n2] = FWD ? ntt_canon<true>(v, q) : csub(shoup_lazy(v, w, ws, q), q);
        });
    __syncthreads();  // the tile's LDS area is reused by the next tile
  }
}

template <bool FWD, int LOGS, int EPW = NTT_EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_blocks_p(NttArgs a, u32 nl, u32 ntiles) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  constexpr int FIRST = FWD ? 0 : Gm::NR - 1;
  using RF = RoundShape<LOGS, LOGR, FIRST>;
  constexpr bool IN_LDS = !FWD, OUT_LDS = FWD;  // coalesce the thread-contiguous side through LDS
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const int n1 = a.log_n - LOGS;
  const u32 tpl = (1u << n1) / PL::SUBS;
  const int sub = PL::sub(), tt = PL::tt();
  u32 t = blockIdx.x;
  if (t >= ntiles) return;
  u64 nx[Gm::R];
  auto fetch = [&](u32 tile) {
    const TileId id = tile_id(tile, nl, tpl);
    const u64* in0 = a.src + (u64)id.limb * a.src_stride + (u64)id.z * a.src_zstride + ((u64)id.pos * PL::SUBS << LOGS);
    if constexpr (IN_LDS) {
#pragma unroll
      for (int k = 0; k < Gm::R; ++k) nx[k] = in0[threadIdx.x + k * THREADS];
    } else {
      const u64* in = in0 + ((u64)sub << LOGS);
#pragma unroll
      for (int u = 0; u < RF::NG; ++u)
#pragma unroll
        for (int i = 0; i < RF::G; ++i) nx[u * RF::G + i] = in[RF::elem(tt, u, i)];
    }
  };
  fetch(t);
  for (; t < ntiles; t += gridDim.x) {
    u64 x[Gm::R];
    if constexpr (IN_LDS) {
#pragma unroll
      for (int k = 0; k < Gm::R; ++k) {
        const int idx = threadIdx.x + k * THREADS;
        lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))] = nx[k];
      }
      __syncthreads();
      lds_get<LOGS, LOGR, FIRST>(lds + sub * Gm::SUB, x, tt);
    } else {
#pragma unroll
      for (int i = 0; i < Gm::R; ++i) x[i] = nx[i];
    }
    if (t + gridDim.x < ntiles) fetch(t + gridDim.x);
    const TileId id = tile_id(t, nl, tpl);
    const u32 mi = a.limb_mod[id.limb];
    const u64 q = a.mods[mi].q;
    const u64 blk0 = (u64)id.pos * PL::SUBS;
    u64* out0 = a.dst + (u64)id.limb * a.dst_stride + (u64)id.z * a.dst_zstride + (blk0 << LOGS);
    u64* out = out0 + ((u64)sub << LOGS);
    sub_transform_regs<FWD, LOGS, LOGR, OUT_LDS>(x, lds + sub * Gm::SUB, tt, a.tw + ((u64)mi << a.log_n),
                                                 (1ull << n1) + blk0 + sub, q,
                                                 [&](int e, u64 v) { out[e] = ntt_canon<FWD>(v, q); });
    if constexpr (OUT_LDS) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < Gm::R; ++k) {
        const int idx = threadIdx.x + k * THREADS;
        out0[idx] = ntt_canon<FWD>(lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))], q);
      }
    }
    __syncthreads();
  }
}

// Experimental: "cols" pass with the (shared) twiddles W[0, S) staged in LDS.
template <bool FWD, int LOGS, int EPW = NTT_EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_cols_twlds(NttArgs a) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, true, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  __shared__ Tw2 tws[Gm::S];
  const int limb = blockIdx.y;
  const u32 mi = a.limb_mod[limb];
  const u64 q = a.mods[mi].q;
  const int n2 = a.log_n - LOGS;
  const int sub = PL::sub(), tt = PL::tt();
  const u64 col = (u64)blockIdx.x * PL::SUBS + sub;
  const u64* in = a.src + (u64)limb * a.src_stride + (u64)blockIdx.z * a.src_zstride + col;
  u64* out = a.dst + (u64)limb * a.dst_stride + (u64)blockIdx.z * a.dst_zstride + col;
  const Tw2* twg = a.tw + ((u64)mi << a.log_n);
  for (int i = threadIdx.x; i < Gm::S; i += THREADS) tws[i] = twg[i];
  u64 w = a.mods[mi].ninv, ws = a.mods[mi].ninvs;
  if (!FWD && a.scale) {
    w = a.scale[2 * (u64)limb];
    ws = a.scale[2 * (u64)limb + 1];
  }
  u64 x[Gm::R];
  {
    constexpr int FIRST = FWD ? 0 : Gm::NR - 1;
    using RS = RoundShape<LOGS, LOGR, FIRST>;
#pragma unroll
    for (int u = 0; u < RS::NG; ++u)
#pragma unroll
      for (int i = 0; i < RS::G; ++i) x[u * RS::G + i] = in[(u64)RS::elem(tt, u, i) << n2];
  }
  __syncthreads();
  sub_transform_regs<FWD, LOGS, LOGR, false>(x, lds + sub * Gm::SUB, tt, tws, 1, q,
      [&](int e, u64 v) {
        out[(u64)e << n2] = FWD ? ntt_canon<true>(v, q) : csub(shoup_lazy(v, w, ws, q), q);
      });
}

// Experimental: persistent "cols" pass, twiddles of the tile's prime staged
// in LDS, next tile (data + twiddles) prefetched into registers.  Workgroup
// g owns the contiguous tile range [g*n/G, (g+1)*n/G).
template <bool FWD, int LOGS, int EPW = NTT_EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_cols_pp(NttArgs a, u32 nl, u32 ntiles) {
  constexpr int LOGR = Radix<LOGS>::LOGR;
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, true, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  constexpr int FIRST = FWD ? 0 : Gm::NR - 1;
  using RF = RoundShape<LOGS, LOGR, FIRST>;
  constexpr int TWPT = (Gm::S + THREADS - 1) / THREADS;  // twiddles per thread
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  __shared__ Tw2 tws[Gm::S];
  const int n2 = a.log_n - LOGS;
  const u32 tpl = (1u << n2) / PL::SUBS;
  const int sub = PL::sub(), tt = PL::tt();
  const u32 t0 = (u32)(((u64)blockIdx.x * ntiles) / gridDim.x);
  const u32 t1 = (u32)(((u64)(blockIdx.x + 1) * ntiles) / gridDim.x);
  if (t0 >= t1) return;
  u64 nx[Gm::R];
  u64 ntw0 = 0, ntw1 = 0;  // one twiddle pair per thread (S <= THREADS)
  static_assert(TWPT == 1, "one twiddle pair per thread");
#define HE_FETCH_COLS(tile)                                                                                  \
  {                                                                                                          \
    const TileId id_ = tile_id(tile, nl, tpl);                                                               \
    const u32 mi_ = ldc(a.limb_mod + id_.limb);                                                              \
    const u64* in_ = a.src + (u64)id_.limb * a.src_stride + (u64)id_.z * a.src_zstride + (u64)id_.pos * PL::SUBS + sub; \
    _Pragma("unroll") for (int u = 0; u < RF::NG; ++u)                                                       \
    _Pragma("unroll") for (int i = 0; i < RF::G; ++i) nx[u * RF::G + i] = in_[(u64)RF::elem(tt, u, i) << n2]; \
    if (threadIdx.x < Gm::S) {                                                                               \
      const Tw2 tv_ = a.tw[((u64)mi_ << a.log_n) + threadIdx.x];                                             \
      ntw0 = tv_.w;                                                                                          \
      ntw1 = tv_.ws;                                                                                         \
    }                                                                                                        \
  }
  HE_FETCH_COLS(t0)
  for (u32 t = t0; t < t1; ++t) {
    u64 x[Gm::R];
#pragma unroll
    for (int i = 0; i < Gm::R; ++i) x[i] = nx[i];
    if (threadIdx.x < Gm::S) tws[threadIdx.x] = Tw2{ntw0, ntw1};
    __syncthreads();
    if (t + 1 < t1) HE_FETCH_COLS(t + 1)
    const TileId id = tile_id(t, nl, tpl);
    const u32 mi = ldc(a.limb_mod + id.limb);
    const u64 q = ldc(&a.mods[mi].q);
    u64* out = a.dst + (u64)id.limb * a.dst_stride + (u64)id.z * a.dst_zstride + (u64)id.pos * PL::SUBS + sub;
    u64 w = ldc(&a.mods[mi].ninv), ws = ldc(&a.mods[mi].ninvs);
    if (!FWD && a.scale) {
      w = ldc(a.scale + 2 * (u64)id.limb);
      ws = ldc(a.scale + 2 * (u64)id.limb + 1);
    }
    sub_transform_regs<FWD, LOGS, LOGR, false>(x, lds + sub * Gm::SUB, tt, tws, 1, q,
        [&](int e, u64 v) {
          out[(u64)e << n2] = FWD ? ntt_canon<true>(v, q) : csub(shoup_lazy(v, w, ws, q), q);
        });
    __syncthreads();
  }
#undef HE_FETCH_COLS
}

}  // namespace he
