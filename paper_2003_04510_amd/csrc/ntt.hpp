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
//                  stage m_loc uses W[m_loc (2^n1 + b) + j].
// Inside a pass each workgroup stages several sub-transforms in LDS; each
// thread holds R = 2^LOGR elements in registers and runs LOGR stages per
// round (radix-2^LOGR), with one LDS exchange between rounds.
//
// The inverse runs the same butterfly network backwards (Gentleman-Sande
// butterflies with TB_invW, stages in reverse order): "blocks" first, then
// "cols", then the factor N^{-1} (optionally merged with a per-limb
// constant).
//
// Lazy ranges (registers and LDS only): forward values live in [0, 4q)
// (Harvey's butterfly), inverse values in [0, 2q).  Every value written to
// global memory is canonical.
#pragma once
#include "modarith.hpp"

namespace he {

template <int LOGS, int LOGR>
struct Geo {
  static constexpr int S = 1 << LOGS;
  static constexpr int R = 1 << LOGR;
  static constexpr int T = S / R;                      // threads per sub-transform
  static constexpr int NR = (LOGS + LOGR - 1) / LOGR;  // register rounds
  static constexpr int SUB = S + (S >> 4) + 1;         // padded LDS stride (words)
  __device__ static __forceinline__ int pad(int e) { return e + (e >> 4); }
};

// One register round: stages st .. st+rr-1 of a 2^LOGS-point sub-transform
// whose elements sit in `tile` (padded).  base: twiddle index multiplier
// (1 for "cols", 2^n1 + b for "blocks").
template <bool FWD, int LOGS, int LOGR, int RD>
__device__ __forceinline__ void ntt_round(u64* tile, int tt, const u64* __restrict__ w,
                                          const u64* __restrict__ ws, u64 base, u64 q) {
  using Gm = Geo<LOGS, LOGR>;
  constexpr int st = RD * LOGR;
  constexpr int rr = (LOGS - st) < LOGR ? (LOGS - st) : LOGR;
  constexpr int G = 1 << rr;
  constexpr int NG = Gm::R / G;
  constexpr int cnt_c = Gm::S >> (st + rr);  // also the element spacing inside a group
  constexpr int span = Gm::S >> st;
  const u64 q2 = q << 1;
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    const int g = tt + u * Gm::T;
    const int blk = g / cnt_c, c = g % cnt_c;
    const int e0 = blk * span + c;
    u64 x[G];
#pragma unroll
    for (int i = 0; i < G; ++i) x[i] = tile[Gm::pad(e0 + i * cnt_c)];
    if constexpr (FWD) {
#pragma unroll
      for (int k = 0; k < rr; ++k) {
        const int half = G >> (k + 1);
        const u64 mloc = 1ull << (st + k);
#pragma unroll
        for (int i = 0; i < G; ++i) {
          if (i & half) continue;
          const u64 idx = mloc * base + ((u64)blk << k) + (u64)(i >> (rr - k));
          const u64 W = w[idx], Ws = ws[idx];
          const u64 X = csub(x[i], q2);
          const u64 Tt = shoup_lazy(x[i + half], W, Ws, q);
          x[i + half] = X - Tt + q2;
          x[i] = X + Tt;
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
          const u64 idx = mloc * base + ((u64)blk << k) + (u64)(i >> (rr - k));
          const u64 W = w[idx], Ws = ws[idx];
          const u64 X = x[i], Y = x[i + half];
          x[i] = csub(X + Y, q2);
          x[i + half] = shoup_lazy(X - Y + q2, W, Ws, q);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < G; ++i) tile[Gm::pad(e0 + i * cnt_c)] = x[i];
  }
}

template <bool FWD, int LOGS, int LOGR, int RD = 0>
__device__ __forceinline__ void ntt_rounds(u64* tile, int tt, const u64* __restrict__ w,
                                           const u64* __restrict__ ws, u64 base, u64 q) {
  constexpr int NR = Geo<LOGS, LOGR>::NR;
  if constexpr (RD < NR) {
    constexpr int ridx = FWD ? RD : NR - 1 - RD;
    ntt_round<FWD, LOGS, LOGR, ridx>(tile, tt, w, ws, base, q);
    __syncthreads();
    ntt_rounds<FWD, LOGS, LOGR, RD + 1>(tile, tt, w, ws, base, q);
  }
}

// Final canonical reduction of a lazy value; the inverse "cols" pass also
// multiplies by (w, ws) = N^{-1} (or N^{-1} times a per-limb constant).
template <bool FWD>
__device__ __forceinline__ u64 ntt_finish(u64 x, u64 q, u64 w, u64 ws) {
  if constexpr (FWD) {
    return csub(csub(x, q << 1), q);
  } else {
    return csub(shoup_lazy(x, w, ws, q), q);
  }
}

// Arguments of one batched transform launch: limb l of the batch reads
// src + l*src_stride, writes dst + l*dst_stride (in place allowed), works
// modulo mods[limb_mod[l]], and (inverse "cols" pass only) multiplies by the
// Shoup pair scale[2l], scale[2l+1] instead of N^{-1} when scale != null.
struct NttArgs {
  const u64* src;
  u64* dst;
  u64 src_stride, dst_stride;
  const u32* limb_mod;
  const ModInfo* mods;
  const u64* tw;   // [nmods][N] W (forward) or invW (inverse)
  const u64* tws;  // Shoup companions
  const u64* scale;
  u64 src_zstride, dst_zstride;  // blockIdx.z selects a polynomial
  u32 log_n;
};

template <bool FWD, int LOGS, int LOGR, int C>
__global__ __launch_bounds__(256) void k_ntt_cols(NttArgs a) {
  using Gm = Geo<LOGS, LOGR>;
  __shared__ u64 lds[C * Gm::SUB];
  const int limb = blockIdx.y;
  const u32 mi = a.limb_mod[limb];
  const u64 q = a.mods[mi].q;
  const u64 N = 1ull << a.log_n;
  const int n2 = a.log_n - LOGS;
  const u64 col0 = (u64)blockIdx.x * C;
  const u64* in = a.src + (u64)limb * a.src_stride + (u64)blockIdx.z * a.src_zstride;
  u64* out = a.dst + (u64)limb * a.dst_stride + (u64)blockIdx.z * a.dst_zstride;
  for (int idx = threadIdx.x; idx < C * Gm::S; idx += blockDim.x) {
    const int c = idx % C, r = idx / C;
    lds[c * Gm::SUB + Gm::pad(r)] = in[col0 + c + ((u64)r << n2)];
  }
  __syncthreads();
  const int sub = threadIdx.x / Gm::T, tt = threadIdx.x % Gm::T;
  ntt_rounds<FWD, LOGS, LOGR>(lds + sub * Gm::SUB, tt, a.tw + (u64)mi * N, a.tws + (u64)mi * N, 1, q);
  u64 w = a.mods[mi].ninv, ws = a.mods[mi].ninvs;
  if (!FWD && a.scale) {
    w = a.scale[2 * (u64)limb];
    ws = a.scale[2 * (u64)limb + 1];
  }
  for (int idx = threadIdx.x; idx < C * Gm::S; idx += blockDim.x) {
    const int c = idx % C, r = idx / C;
    out[col0 + c + ((u64)r << n2)] = ntt_finish<FWD>(lds[c * Gm::SUB + Gm::pad(r)], q, w, ws);
  }
}

template <bool FWD, int LOGS, int LOGR, int B>
__global__ __launch_bounds__(256) void k_ntt_blocks(NttArgs a) {
  using Gm = Geo<LOGS, LOGR>;
  __shared__ u64 lds[B * Gm::SUB];
  const int limb = blockIdx.y;
  const u32 mi = a.limb_mod[limb];
  const u64 q = a.mods[mi].q;
  const u64 N = 1ull << a.log_n;
  const int n1 = a.log_n - LOGS;
  const u64 blk0 = (u64)blockIdx.x * B;
  const u64* in = a.src + (u64)limb * a.src_stride + (u64)blockIdx.z * a.src_zstride + (blk0 << LOGS);
  u64* out = a.dst + (u64)limb * a.dst_stride + (u64)blockIdx.z * a.dst_zstride + (blk0 << LOGS);
  for (int idx = threadIdx.x; idx < B * Gm::S; idx += blockDim.x)
    lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))] = in[idx];
  __syncthreads();
  const int sub = threadIdx.x / Gm::T, tt = threadIdx.x % Gm::T;
  const u64 base = (1ull << n1) + blk0 + sub;
  ntt_rounds<FWD, LOGS, LOGR>(lds + sub * Gm::SUB, tt, a.tw + (u64)mi * N, a.tws + (u64)mi * N, base, q);
  for (int idx = threadIdx.x; idx < B * Gm::S; idx += blockDim.x)
    out[idx] = csub(csub(lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))], FWD ? (q << 1) : ~0ull), q);
}

}  // namespace he
