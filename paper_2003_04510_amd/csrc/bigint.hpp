// Device kernels of the paper's non-RNS HE Mul (Sec. III, Fig. 2): big-integer
// polynomials with power-of-two moduli, multiplied through RNS (CRT), NTT,
// element-wise products, inverse NTT and RNS-to-BigInt conversion (iCRT).
//
// Layout: a big-integer polynomial is word-major, [W][N] little-endian
// 64-bit words (word w of coefficient n at w*N + n), so a wavefront's lanes
// (consecutive coefficients) read consecutive addresses.  RNS form is
// limb-major, [np][N].
//
//   k_big_crt    BigInt -> RNS in matrix form (Sec. IV-A, "GPU-C") on the
//                int8 matrix cores (v_mfma_i32_16x16x32_i8): x mod p_i =
//                sum_h u_h [2^(8h)]_{p_i} over the bytes u_h of x, with
//                rows = coefficients, k = bytes (offset binary u - 128) and
//                columns = (prime, digit) for the balanced base-256 digits
//                of the constants; per (coefficient, prime) the digit
//                columns are recombined in 128 bits and reduced once.
//   k_big_mul    element-wise products of NTT-form limbs.
//   k_big_icrt   RNS -> BigInt in matrix form (Algorithm 6), also an int8
//                matrix-core product: with y_i = [x_i (M/p_i)^-1]_{p_i}
//                (folded into the inverse NTT's scale), X = sum_i y_i (M/p_i)
//                - k M, k = round(sum_i y_i / p_i) in FP64, only modulo
//                2^(32 C): k = (prime, byte of y), columns = byte positions,
//                B a Toeplitz expansion of the balanced bytes of M/p_i staged
//                per 16-column tile in LDS; byte columns are folded four at a
//                time into 32-bit words and carried serially per
//                coefficient.  The output is a bit field of X: bits
//                [shift, shift + outbits) with optional round-half-up at bit
//                shift - 1 (region 2's shift by log Q).
//   k_big_finish the additions of HE Mul (c3) and the optional rescale by 2^logp.
#pragma once
#include "modarith.hpp"

namespace he {
namespace big {

constexpr int MF_THREADS = 256;                // 4 wavefronts of 16 rows (coefficients) each
constexpr int ICRT_THREADS = MF_THREADS;
constexpr int FIN_THREADS = 256;
constexpr int WMAX = 19;                       // words of a ciphertext coefficient (log Q <= 1216)
constexpr int CRT_KBMAX = 10;                  // 32-byte k-blocks of a CRT input (2 log Q bits)
constexpr int ICRT_KBMAX = 16;                 // k-blocks of the iCRT (4 primes each, np <= 64)

typedef int v4i __attribute__((ext_vector_type(4)));

// 16x16 int32 tile += A (16 x 32 int8) * B (32 x 16 int8).  Lane l supplies
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] as byte j of a
// 64-bit operand and receives D[4 (l / 16) + j][l % 16] in element j.
__device__ __forceinline__ v4i mfma_i8(long a, long b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x32_i8(a, b, c, 0, 0, 0);
}

// Offset binary: the bytes u of a word as signed int8 values u - 128.
__device__ __forceinline__ long offset_bytes(u64 w) { return (long)(w ^ 0x8080808080808080ull); }

// One CRT job: src [W][N] -> dst [np][N].
struct CrtArgs {
  const u64* src[4];
  u64* dst[4];
  const ModInfo* mods;  // [np]
  const u64* B;         // [4 kbmax][ncols]: word kw of column 8i+b: bytes j = digit b of [2^(8 (8kw+j))]_{p_i}
  const u64* adj;       // [np2]: ([128 sum_h c_{i,h}] - [2^80]) mod p_i
  u32 np, W, kb, ncols, log_n;
};

// x mod p_i as a matrix product (the matrix form of CRT): with x = sum_h u_h
// 2^(8h) (bytes) and c_{i,h} = [2^(8h)]_{p_i} = sum_b t_{i,h,b} 2^(8b)
// (balanced signed digits), V_i = sum_b 2^(8b) sum_h u_h t_{i,h,b} = sum_h u_h
// c_{i,h} == x (mod p_i).  The inner sums are an int8 GEMM on the matrix
// cores: rows = coefficients, k = bytes h, columns = (prime, digit).  The
// data enter as offset binary (u_h - 128); the correction 128 sum_h c_{i,h}
// is the per-prime constant adj.  Items: (job, 64 coefficients); each wave
// owns 16 coefficients and all the job's primes, four primes (two column
// tiles) per step so that every lane finishes one (coefficient, prime).
__global__ __launch_bounds__(MF_THREADS) void k_big_crt(CrtArgs a) {
  __shared__ int zs[MF_THREADS / 64][16][33];
  const u32 lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const u64 N = 1ull << a.log_n;
  const u32 job = blockIdx.y;
  const u64 n0 = (u64)blockIdx.x * (MF_THREADS / 4) + wave * 16;
  const u32 r = lane & 15, g = lane >> 4;
  // A fragments: word 4 kb + g of coefficient n0 + r
  long A[CRT_KBMAX];
  const auto src = gbl(a.src[job] + n0 + r);
#pragma unroll
  for (int kb = 0; kb < CRT_KBMAX; ++kb) {
    const u32 w = 4 * kb + g;
    A[kb] = (u32)kb < a.kb ? offset_bytes(w < a.W ? src[(u64)w * N] : 0) : 0;
  }
  const auto dst = gbl(a.dst[job]);
  const auto Bg = gbl(a.B + (u64)g * a.ncols + r);
  const u32 steps = (a.np + 3) / 4;
  for (u32 cp = 0; cp < steps; ++cp) {
    // this lane's prime: its constants are loaded ahead of the products
    const u32 i = 4 * cp + g, ic = min(i, a.np - 1);
    const ModInfo m = a.mods[ic];
    const u64 adj = a.adj[ic];
    v4i acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    const u32 c0 = 32 * cp;
#pragma unroll
    for (int kb = 0; kb < CRT_KBMAX; ++kb)
      if ((u32)kb < a.kb) {
        const u64 off = (u64)(4 * kb) * a.ncols + c0;
        acc0 = mfma_i8(A[kb], (long)Bg[off], acc0);
        acc1 = mfma_i8(A[kb], (long)Bg[off + 16], acc1);
      }
    // D rows 4g + j; columns c0 + r (acc0) and c0 + 16 + r (acc1)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      zs[wave][4 * g + j][r] = acc0[j];
      zs[wave][4 * g + j][16 + r] = acc1[j];
    }
    lds_wave_sync();
    // lane: coefficient r, prime 4 cp + g (digits at columns 8 g .. 8 g + 7)
    if (i < a.np) {
      const int* z = &zs[wave][r][8 * g];
      // V = sum_b 2^(8b) z_b, |V| < 2^79; U = V + 2^80 > 0
      long long lo = 0, hi = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) lo += (long long)z[b] << (8 * b);
#pragma unroll
      for (int b = 0; b < 4; ++b) hi += (long long)z[4 + b] << (8 * b);
      typedef __int128 i128;
      const i128 v = (i128)lo + ((i128)hi << 32) + ((i128)1 << 80);
      U128 u;
      u.lo = (u64)v;
      u.hi = (u64)(v >> 64);
      dst[(u64)i * N + n0 + r] = addmod(reduce128(u, m), adj, m.q);
    }
    lds_wave_sync();
  }
}

// Region 1's products in NTT form from the four operand transforms
// t = (ax1, ax2, bx1, bx2) [4][np][N]: slot 0 <- (ax1+bx1)(ax2+bx2),
// slot 1 <- ax1 ax2, slot 2 <- bx1 bx2 (each element read before written).
// The Karatsuba sums are taken in RNS, without the reduction mod q: the
// product differs from HEAAN's by a multiple of q, and the result is taken
// mod q (the region-1 primes cover the doubled operands).
__global__ __launch_bounds__(256) void k_big_mul_r1(u64* t, const ModInfo* mods, u32 np, u32 log_n) {
  const u64 N = 1ull << log_n;
  const u64 e = (u64)blockIdx.x * 256 + threadIdx.x;
  const u32 i = (u32)(e >> log_n);
  if (i >= np) return;
  const ModInfo m = ldc(mods + uniform(i));
  const u64 L = (u64)np * N, off = e;
  const auto p = gbl(t);
  const u64 a1 = p[off], a2 = p[L + off], b1 = p[2 * L + off], b2 = p[3 * L + off];
  p[off] = mulmod(addmod(a1, b1, m.q), addmod(a2, b2, m.q), m);
  p[L + off] = mulmod(a1, a2, m);
  p[2 * L + off] = mulmod(b1, b2, m);
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

struct IcrtArgs {
  const u64* src;        // [njobs][np][N], y_i (canonical)
  u64* dst;              // [njobs][W][N] words
  const double* pinv;    // [np] fl(1/p_i)
  const u64* B;          // [64][Pc]: byte j = digit P - j of (M/p_i) mod 2^(32 Ct) (balanced, zero outside)
  const long long* CW;   // [Ct]: offset correction of word column m, sum_b 128 colsum[4m+b] 2^(8b)
  const u32* negM;       // [Ct]: words of -M mod 2^(32 Ct)
  u32 np, kb, Pc, C, shift, round, outbits, W, log_n;
};

// X = sum_i y_i (M/p_i) - k M modulo 2^(32 C) as a matrix product (the
// matrix form of iCRT, Algorithm 6): with y_i = sum_a y_{i,a} 2^(8a) and
// (M/p_i) = sum_b t_{i,b} 2^(8b), byte column P of the product is
// Z_P = sum_{i,a} y_{i,a} t_{i,P-a}, an int8 GEMM on the matrix cores with
// k = (prime, byte of y) and a Toeplitz B.  The data enter as offset binary
// (the correction is CW); the byte columns are folded four at a time into
// 32-bit words and carried serially per coefficient.  The output is the bit
// field [shift, shift + outbits) of X with optional round-half-up at bit
// shift - 1.  Items: (job, 64 coefficients), 16 per wave; the B tile of a
// column tile is staged in LDS for the workgroup.
__global__ __launch_bounds__(MF_THREADS) void k_big_icrt(IcrtArgs a) {
  __shared__ u64 bs[2][64][16];
  __shared__ int zs[MF_THREADS / 64][16][17];
  const u32 lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const u64 N = 1ull << a.log_n;
  const u32 job = blockIdx.y;
  const u64 n0 = (u64)blockIdx.x * (MF_THREADS / 4) + wave * 16;
  const u32 r = lane & 15, g = lane >> 4;
  const u32 tiles = (a.C + 3) / 4;
  // B tile ct: 1024 fragments, entry e = i * 16 + column
  u64 pf[4];
  const auto fetch = [&](u32 ct) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const u32 idx = threadIdx.x + e * MF_THREADS;
      pf[e] = a.B[(u64)(idx >> 4) * a.Pc + 16 * ct + (idx & 15)];
    }
  };
  const auto stage = [&](u32 buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const u32 idx = threadIdx.x + e * MF_THREADS;
      bs[buf][idx >> 4][idx & 15] = pf[e];
    }
  };
  fetch(0);
  const auto src = gbl(a.src + (u64)job * a.np * N + n0 + r);
  long A[ICRT_KBMAX];
  double s = 0.0;
#pragma unroll
  for (int kb = 0; kb < ICRT_KBMAX; ++kb) {
    const u32 i = 4 * kb + g;
    const u64 y = ((u32)kb < a.kb && i < a.np) ? src[(u64)i * N] : 0;
    if (i < a.np) s += (double)y * ldc(a.pinv + i);
    A[kb] = offset_bytes(y);
  }
  stage(0);
  // sum_i y_i / p_i over the four lane groups of this row
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  // sum y_i / p_i = k + X / M with |X| / M < 1/4: round to nearest
  const long long k = __double2int_rn(s);
  const auto out = reinterpret_cast<gptr<u32>>(gbl(a.dst + (u64)job * a.W * N + n0 + r));
  const u32 cs = a.shift >> 5, sh = a.shift & 31;
  const u32 ocols = (a.outbits + 31) >> 5;
  const u32 rcol = a.round ? (a.shift - 1) >> 5 : ~0u;
  const long long rval = a.round ? 1ll << ((a.shift - 1) & 31) : 0;
  const bool owner = lane < 16;  // lane r carries row r
  const auto emit = [&](u32 m, u32 v) {
    if (m >= ocols) return;
    if (m == ocols - 1 && (a.outbits & 31)) v &= (1u << (a.outbits & 31)) - 1;
    out[((u64)(m >> 1) * N) * 2 + (m & 1)] = v;
  };
  if (owner)
    for (u32 m = ocols; m < 2 * a.W; ++m) out[((u64)(m >> 1) * N) * 2 + (m & 1)] = 0;
  long long cy = 0;
  u32 prev = 0;
  lds_barrier();
  for (u32 ct = 0; ct < tiles; ++ct) {
    const u32 buf = ct & 1;
    if (ct + 1 < tiles) fetch(ct + 1);  // in flight during this tile
    v4i acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < ICRT_KBMAX; kb += 2) {
      if ((u32)kb < a.kb) acc0 = mfma_i8(A[kb], (long)bs[buf][4 * kb + g][r], acc0);
      if ((u32)kb + 1 < a.kb) acc1 = mfma_i8(A[kb + 1], (long)bs[buf][4 * kb + 4 + g][r], acc1);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) zs[wave][4 * g + j][r] = acc0[j] + acc1[j];
    lds_wave_sync();
    if (owner) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const u32 m = 4 * ct + q;  // 32-bit word column
        if (m >= a.C) break;
        const int* z = &zs[wave][r][4 * q];
        long long w = (long long)z[0] + ((long long)z[1] << 8) + ((long long)z[2] << 16) +
                      ((long long)z[3] << 24);
        w += ldc(a.CW + m) + k * (long long)ldc(a.negM + m) + cy;
        if (m == rcol) w += rval;
        const u32 col = (u32)w;
        cy = w >> 32;  // arithmetic: the carry may be negative
        if (sh == 0) {
          if (m >= cs) emit(m - cs, col);
        } else if (m >= cs + 1) {
          emit(m - cs - 1, (prev >> sh) | (col << (32 - sh)));
        }
        prev = col;
      }
    }
    lds_wave_sync();
    // buffer buf ^ 1 was last read in tile ct - 1, before the previous barrier
    if (ct + 1 < tiles) stage(buf ^ 1);
    lds_barrier();
  }
  if (owner && sh && a.C >= cs + 1) emit(a.C - cs - 1, prev >> sh);
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
