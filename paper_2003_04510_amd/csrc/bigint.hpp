// Device kernels of the paper's non-RNS HE Mul (Sec. III, Fig. 2): big-integer
// polynomials with power-of-two moduli, multiplied through RNS (CRT), NTT,
// element-wise products, inverse NTT and RNS-to-BigInt conversion (iCRT).
//
// Layout: a big-integer polynomial is word-major, [W][N] little-endian
// 64-bit words (word w of coefficient n at w*N + n), so a wavefront's lanes
// (consecutive coefficients) read consecutive addresses.  RNS form is
// limb-major, [np][N].
//
//   k_big_crt    BigInt -> RNS in matrix form (Sec. IV-A, "GPU-C"): the
//                coefficient is cut into 28-bit digits d_h and
//                x mod p = sum_h d_h [2^(28h)]_p, accumulated as two 64-bit
//                sums of 28x30-bit products (no carries for <= 64 digits),
//                one reduction per prime.
//   k_big_mul    element-wise products of NTT-form limbs.
//   k_big_icrt   RNS -> BigInt in matrix form (Algorithm 6): with
//                y_i = [x_i (M/p_i)^-1]_{p_i} (folded into the inverse NTT's
//                scale), X = sum_i y_i (M/p_i) - k M, k = round(sum_i y_i/p_i)
//                (the centred value), only modulo 2^(32 C): the products of
//                y (two 32-bit halves) with the 32-bit words of (M/p_i) are
//                summed column by column (product scanning, eight columns
//                per pass over the primes, y staged in LDS) in 64 bits plus
//                a 32-bit carry count, so no partial product is ever stored.
//                The output is a bit field of X: bits [shift, shift + outbits)
//                with optional round-half-up at bit shift - 1 (region 2's
//                shift by log Q).
//   k_big_finish the additions of HE Mul (c3) and the optional rescale by 2^logp.
#pragma once
#include "modarith.hpp"

namespace he {
namespace big {

constexpr int CRT_THREADS = 256, CRT_PG = 8;   // primes per work item
constexpr int DIG = 28;                        // CRT digit width
constexpr int DIG_BLOCK = 44;                  // digits summed before a reduction (< 64)
constexpr int ICRT_THREADS = 64;
constexpr int FIN_THREADS = 256;
constexpr int WMAX = 19;                       // words of a ciphertext coefficient (log Q <= 1216)

// One CRT job: src (+ src2, summed modulo 2^bits) -> dst [np][N].
struct CrtJob {
  const u64* a;
  const u64* b;
  u64* dst;
};

struct CrtArgs {
  CrtJob job[6];
  const ModInfo* mods;  // [np]
  const u32* cc;        // [np][ndmax][2]: 30-bit halves of 2^(28h) mod p_i
  u32 np, W, bits, nd, ndmax, log_n;
};

// Words of one coefficient, summed with a second operand modulo 2^bits.
template <int WM>
__device__ __forceinline__ void load_words(const CrtArgs& a, const CrtJob& J, u64 n, u64 (&w)[WM + 1]) {
  const u64 N = 1ull << a.log_n;
  const auto pa = gbl(J.a + n);
#pragma unroll
  for (int k = 0; k < WM; ++k) w[k] = (u32)k < a.W ? pa[(u64)k * N] : 0;
  w[WM] = 0;
  if (J.b) {
    const auto pb = gbl(J.b + n);
    u64 cy = 0;
#pragma unroll
    for (int k = 0; k < WM; ++k) {
      const u64 y = (u32)k < a.W ? pb[(u64)k * N] : 0;
      const u64 s = w[k] + y;
      const u64 c1 = s < y ? 1 : 0;
      w[k] = s + cy;
      cy = c1 + (w[k] < cy ? 1 : 0);
    }
  }
#pragma unroll
  for (int k = 0; k < WM; ++k) {  // mod 2^bits
    const int lo = 64 * k;
    if (lo >= (int)a.bits) w[k] = 0;
    else if (lo + 64 > (int)a.bits) w[k] &= (1ull << (a.bits - lo)) - 1;
  }
}

// Items: (job, coefficient chunk, prime group), prime group fastest so the
// groups of a chunk read its words while they are in L2.
template <int WM>
__global__ __launch_bounds__(CRT_THREADS) void k_big_crt(CrtArgs a) {
  constexpr int ND = (64 * WM + DIG - 1) / DIG;
  const u32 ngrp = (a.np + CRT_PG - 1) / CRT_PG;
  const u32 grp = blockIdx.x % ngrp, chunk = blockIdx.x / ngrp;
  const CrtJob J = a.job[blockIdx.y];
  const u64 n = (u64)chunk * CRT_THREADS + threadIdx.x;
  const u64 N = 1ull << a.log_n;
  u64 w[WM + 1];
  load_words<WM>(a, J, n, w);
  u32 d[ND];
#pragma unroll
  for (int h = 0; h < ND; ++h) {
    const int bit = DIG * h, j = bit >> 6, off = bit & 63;
    u64 v = w[j] >> off;
    if (off + DIG > 64) v |= w[j + 1] << (64 - off);
    d[h] = (u32)v & ((1u << DIG) - 1);
  }
  const u32 i0 = grp * CRT_PG, i1 = min(a.np, i0 + CRT_PG);
  for (u32 i = i0; i < i1; ++i) {
    const ModInfo m = ldc(a.mods + i);
    const u32* C = a.cc + (u64)i * a.ndmax * 2;
    u64 r = 0;
#pragma unroll
    for (int h0 = 0; h0 < ND; h0 += DIG_BLOCK) {
      u64 s0 = 0, s1 = 0;
#pragma unroll
      for (int h = h0; h < h0 + DIG_BLOCK && h < ND; ++h) {
        const bool use = (u32)h < a.nd;
        const u32 c0 = use ? ldc(C + 2 * h) : 0u, c1 = use ? ldc(C + 2 * h + 1) : 0u;
        s0 += (u64)d[h] * c0;
        s1 += (u64)d[h] * c1;
      }
      // s0 + s1 2^30 as a 128-bit value
      U128 v;
      v.lo = s0 + (s1 << 30);
      v.hi = (s1 >> 34) + (v.lo < s0 ? 1 : 0);
      r = addmod(r, reduce128(v, m), m.q);
    }
    gbl(J.dst)[(u64)i * N + n] = r;
  }
}

// out_k[i] = x_k[i] * y_k[i] mod p_i for k < nk, i < np.
struct MulArgs {
  const u64* x[3];
  const u64* y[3];
  u64* out[3];
  const ModInfo* mods;
  u32 np, nk, log_n;
};

__global__ __launch_bounds__(256) void k_big_mul(MulArgs a) {
  const u64 N = 1ull << a.log_n;
  const u64 e = (u64)blockIdx.x * 256 + threadIdx.x;  // element within limb set
  const u32 i = (u32)(e >> a.log_n);
  if (i >= a.np) return;
  const ModInfo m = ldc(a.mods + uniform(i));
  const u64 off = (u64)i * N + (e & (N - 1));
  for (u32 k = 0; k < a.nk; ++k) {
    const u64 xv = gbl(a.x[k])[off], yv = gbl(a.y[k])[off];
    gbl(a.out[k])[off] = mulmod(xv, yv, m);
  }
}

constexpr int ICRT_NPMAX = 64, ICRT_CT = 8;  // primes; columns per tile

struct IcrtArgs {
  const u64* src;       // [njobs][np][N], y_i (canonical)
  u64* dst;             // [njobs][W][N] words
  const double* pinv;   // [np] fl(1/p_i)
  const u32* T;         // [np][Ct + 1 + ICRT_CT]: 0, words 0 .. Ct-1 of (M/p_i) mod 2^(32 Ct), zeros
  const u32* negM;      // [Ct]: words of -M mod 2^(32 Ct)
  u32 np, Ct, C, shift, round, outbits, W, log_n;
};

__global__ __launch_bounds__(ICRT_THREADS) void k_big_icrt(IcrtArgs a) {
  __shared__ u32 ys[2][ICRT_NPMAX][ICRT_THREADS];
  const u64 N = 1ull << a.log_n;
  const u32 tid = threadIdx.x;
  const u64 n = (u64)blockIdx.x * ICRT_THREADS + tid;
  const u32 job = blockIdx.y;
  const auto src = gbl(a.src + (u64)job * a.np * N + n);
  double s = 0.0;
  for (u32 i = 0; i < a.np; ++i) {
    const u64 y = src[(u64)i * N];
    ys[0][i][tid] = (u32)y;
    ys[1][i][tid] = (u32)(y >> 32);
    s += (double)y * ldc(a.pinv + i);
  }
  // sum y_i / p_i = k + X / M with |X| / M < 1/4: round to nearest
  const u32 k = (u32)__double2int_rn(s);
  const auto out = reinterpret_cast<gptr<u32>>(gbl(a.dst + (u64)job * a.W * N + n));
  const u32 cs = a.shift >> 5, sh = a.shift & 31;
  const u32 ocols = (a.outbits + 31) >> 5;
  const u32 rcol = a.round ? (a.shift - 1) >> 5 : ~0u, rbit = (a.shift - 1) & 31;
  // output column m of 32 bits -> word m/2, half m%2 (little-endian halves)
  const auto emit = [&](u32 m, u32 v) {
    if (m >= ocols) return;
    if (m == ocols - 1 && (a.outbits & 31)) v &= (1u << (a.outbits & 31)) - 1;
    out[((u64)(m >> 1) * N) * 2 + (m & 1)] = v;
  };
  for (u32 m = ocols; m < 2 * a.W; ++m) out[((u64)(m >> 1) * N) * 2 + (m & 1)] = 0;
  // Columns c0 .. c0+CT-1 of X: S_j = sum_i y_i.lo T_i[c] + y_i.hi T_i[c-1],
  // 64-bit sums with a count of their carries.  Only this thread's LDS
  // entries are read, so no barrier is needed.
  u64 cy = 0;  // carry into the next column (< 2^40)
  u32 prev = 0;
  const u32 row = a.Ct + 1 + ICRT_CT;  // a tile's last reads stay inside the row
  for (u32 c0 = 0; c0 < a.C; c0 += ICRT_CT) {
    u64 S[ICRT_CT];
    u32 Sh[ICRT_CT];
#pragma unroll
    for (int j = 0; j < ICRT_CT; ++j) S[j] = 0, Sh[j] = 0;
    for (u32 i = 0; i < a.np; ++i) {
      const u32 y0 = ys[0][i][tid], y1 = ys[1][i][tid];
      const u32* Ti = a.T + (u64)i * row + c0;  // Ti[j] = word c0 + j - 1
      u32 t[ICRT_CT + 1];
#pragma unroll
      for (int j = 0; j <= ICRT_CT; ++j) t[j] = ldc(Ti + j);
#pragma unroll
      for (int j = 0; j < ICRT_CT; ++j) {
        u64 p = (u64)y0 * t[j + 1];
        S[j] += p;
        Sh[j] += S[j] < p ? 1u : 0u;
        p = (u64)y1 * t[j];
        S[j] += p;
        Sh[j] += S[j] < p ? 1u : 0u;
      }
    }
#pragma unroll
    for (int j = 0; j < ICRT_CT; ++j) {
      const u32 c = c0 + j;
      if (c >= a.C) break;
      u64 p = (u64)k * ldc(a.negM + c);
      if (c == rcol) p += 1ull << rbit;
      p += cy;
      S[j] += p;
      Sh[j] += S[j] < p ? 1u : 0u;
      const u32 col = (u32)S[j];
      cy = (S[j] >> 32) | ((u64)Sh[j] << 32);
      if (sh == 0) {
        if (c >= cs) emit(c - cs, col);
      } else if (c >= cs + 1) {
        emit(c - cs - 1, (prev >> sh) | (col << (32 - sh)));
      }
      prev = col;
    }
  }
  if (sh && a.C >= cs + 1) emit(a.C - cs - 1, prev >> sh);
}

// c3 = (ks_b + bxbx, ks_a + axbx - axax - bxbx) mod 2^logq, then optionally
// round(c3 / 2^logp) mod 2^(logq - logp).  One thread per coefficient, words
// streamed low to high with carries.
struct FinArgs {
  const u64* ks;   // [2][W][N]: ks_b, ks_a
  const u64* r1;   // [3][W][N]: axbx, axax, bxbx
  u64* out;        // [2][W][N]
  u32 W, logq, logp, log_n;
};

__global__ __launch_bounds__(FIN_THREADS) void k_big_finish(FinArgs a) {
  typedef unsigned __int128 u128;
  const u64 N = 1ull << a.log_n;
  const u64 n = (u64)blockIdx.x * FIN_THREADS + threadIdx.x;
  const u32 u = blockIdx.y;  // 0: bx, 1: ax
  const u64 WN = (u64)a.W * N;
  const auto ks = gbl(a.ks + u * WN + n);
  const auto axbx = gbl(a.r1 + n), axax = gbl(a.r1 + WN + n), bxbx = gbl(a.r1 + 2 * WN + n);
  const auto out = gbl(a.out + u * WN + n);
  const u32 obits = a.logq - a.logp;
  const auto masked = [&](u32 w, u64 v, u32 bits) -> u64 {
    const u32 lo = 64 * w;
    if (lo >= bits) return 0;
    if (lo + 64 > bits) return v & ((1ull << (bits - lo)) - 1);
    return v;
  };
  // value words v_w, built low to high
  u128 carry = 0;   // ax: adds ~axax + ~bxbx + 2 (two's complement); bx: one addition
  u64 prev = 0;
  u64 rc = a.logp ? (1ull << (a.logp - 1)) : 0;  // rounding addend, then its carry
  for (u32 w = 0; w < a.W; ++w) {
    u128 t = carry + ks[(u64)w * N];
    if (u) {
      t += axbx[(u64)w * N];
      t += (u64)~axax[(u64)w * N];
      t += (u64)~bxbx[(u64)w * N];
      if (w == 0) t += 2;
    } else {
      t += bxbx[(u64)w * N];
    }
    u64 v = (u64)t;
    carry = t >> 64;
    v = masked(w, v, a.logq);
    if (!a.logp) {
      out[(u64)w * N] = v;
      continue;
    }
    // rounding: v + 2^(logp-1), carried up through the words
    const u64 vr = v + rc;
    rc = vr < v ? 1 : 0;
    if (w) out[(u64)(w - 1) * N] = masked(w - 1, (prev >> a.logp) | (vr << (64 - a.logp)), obits);
    prev = vr;
  }
  if (a.logp) out[(u64)(a.W - 1) * N] = masked(a.W - 1, prev >> a.logp, obits);
}

}  // namespace big
}  // namespace he
