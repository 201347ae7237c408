// Device kernels of the steps around HE Mul (Sec. III-A, III-B): CKKS
// encoding of complex slots into integer coefficients (an FP64 FFT over the
// odd powers of zeta = exp(i pi / N)) and HE Add.
//
// Encoding: slot j sits at zeta^{5^j mod 2N}; with V[t] the value wanted at
// zeta^{2t+1} (scale z_j there and its conjugate at the conjugate root), the
// coefficients are m_k = Re(zeta^{-k} (1/N) sum_t V[t] e^{-2 pi i t k / N}),
// rounded to nearest (ties to even).  The FFT is radix-2, decimation in time
// after a bit-reversal permutation, one launch per stage (the encoding is
// not on the HE Mul path).
#pragma once
#include "modarith.hpp"

namespace he {
namespace enc {

constexpr int THREADS = 256;

struct cplx {
  double re, im;
};

// V = 0 except at the slots' roots; written in bit-reversed order for the
// in-place FFT that follows.  One thread per slot j < N/2.
__global__ __launch_bounds__(THREADS) void k_enc_scatter(const double* z, u32 n, double scale, cplx* V,
                                                         u32 log_n) {
  const u64 N = 1ull << log_n;
  const u64 j = (u64)blockIdx.x * THREADS + threadIdx.x;
  if (j >= N / 2) return;
  // 5^j mod 2N by square-and-multiply
  u64 e = 1, b = 5, k = j;
  const u64 mask = 2 * N - 1;
  while (k) {
    if (k & 1) e = (e * b) & mask;
    b = (b * b) & mask;
    k >>= 1;
  }
  double re = 0.0, im = 0.0;
  if (j < n) {
    re = scale * z[2 * j];
    im = scale * z[2 * j + 1];
  }
  const u32 t0 = (u32)((e - 1) / 2), t1 = (u32)((2 * N - e - 1) / 2);
  const u32 r0 = __brev(t0) >> (32 - log_n), r1 = __brev(t1) >> (32 - log_n);
  V[r0] = cplx{re, im};
  V[r1] = cplx{re, -im};
}

// One radix-2 stage: butterflies of span h = 2^(s-1) with w = e^{sign i pi j / h}
// (sign -1: forward transform, +1: the unnormalized inverse).
__global__ __launch_bounds__(THREADS) void k_fft_stage(cplx* V, u32 s, u32 log_n, double sign) {
  const u64 b = (u64)blockIdx.x * THREADS + threadIdx.x;
  if (b >= (1ull << (log_n - 1))) return;
  const u64 h = 1ull << (s - 1);
  const u64 j = b & (h - 1), i0 = ((b >> (s - 1)) << s) + j, i1 = i0 + h;
  double sn, cs;
  sincospi(sign * (double)j / (double)h, &sn, &cs);
  const cplx x0 = V[i0], x1 = V[i1];
  const double tr = x1.re * cs - x1.im * sn, ti = x1.re * sn + x1.im * cs;
  V[i0] = cplx{x0.re + tr, x0.im + ti};
  V[i1] = cplx{x0.re - tr, x0.im - ti};
}

// m_k = rint(Re(x_k zeta^{-k}) / N).
__global__ __launch_bounds__(THREADS) void k_enc_finish(const cplx* X, int64_t* m, u32 log_n) {
  const u64 N = 1ull << log_n;
  const u64 k = (u64)blockIdx.x * THREADS + threadIdx.x;
  if (k >= N) return;
  double sn, cs;
  sincospi(-(double)k / (double)N, &sn, &cs);
  const cplx x = X[k];
  const double v = (x.re * cs - x.im * sn) / (double)N;
  m[k] = (int64_t)rint(v);
}

// Decoding, step 1: the centred integer of each coefficient from its level
// residues (mixed radix with balanced digits: x = sum_i d_i W_i,
// W_i = q_0 ... q_{i-1}, d_i in (-q_i/2, q_i/2], Garner's recurrence), as a
// double (the sum of the nonzero terms, largest first), times zeta^k, written
// at the bit-reversed index for the inverse FFT.  Digits that reach a
// weight beyond the double range give an infinite value (the coefficient
// is then no message).  One thread per coefficient.
struct DecArgs {
  const u64* m;          // [level][N] residues
  const ModInfo* mods;
  const u64* wmod;       // [level][level]: [W_j]_{q_i} (j < i) at i * level + j; [W_i^-1]_{q_i} at i * level + i
  const double* wd;      // [level]: W_i as a double (inf past the range)
  cplx* V;
  u32 level, log_n;
};

__global__ __launch_bounds__(THREADS) void k_dec_crt(DecArgs a) {
  const u64 N = 1ull << a.log_n;
  const u64 k = (u64)blockIdx.x * THREADS + threadIdx.x;
  if (k >= N) return;
  constexpr int LMAX = 64;
  int64_t d[LMAX];  // balanced digits (|d| < 2^59)
  double v = 0.0;
  for (u32 i = 0; i < a.level; ++i) {
    const ModInfo m = a.mods[i];
    // t = sum_{j<i} d_j W_j mod q_i
    u64 t = 0;
    for (u32 j = 0; j < i; ++j) {
      const u64 rj = (u64)(d[j] < 0 ? -d[j] : d[j]) % m.q;
      const u64 dj = (d[j] < 0 && rj) ? m.q - rj : rj;
      t = addmod(t, mulmod(dj, a.wmod[(u64)i * a.level + j], m), m.q);
    }
    const u64 x = a.m[(u64)i * N + k];
    u64 di = mulmod(submod(x, t, m.q), a.wmod[(u64)i * a.level + i], m);
    d[i] = 2 * di > m.q ? (int64_t)di - (int64_t)m.q : (int64_t)di;
  }
  for (int i = (int)a.level - 1; i >= 0; --i)
    if (d[i]) v += (double)d[i] * a.wd[i];
  double sn, cs;
  sincospi((double)k / (double)N, &sn, &cs);
  const u32 r = __brev((u32)k) >> (32 - a.log_n);
  a.V[r] = cplx{v * cs, v * sn};
}

// Decoding, step 2: slot j = V[(5^j - 1) / 2] / scale (V[t] = m(zeta^(2t+1))).
__global__ __launch_bounds__(THREADS) void k_dec_gather(const cplx* V, u32 n, double scale, double* z, u32 log_n) {
  const u64 N = 1ull << log_n;
  const u64 j = (u64)blockIdx.x * THREADS + threadIdx.x;
  if (j >= n) return;
  u64 e = 1, b = 5, kk = j;
  const u64 mask = 2 * N - 1;
  while (kk) {
    if (kk & 1) e = (e * b) & mask;
    b = (b * b) & mask;
    kk >>= 1;
  }
  const cplx x = V[(e - 1) / 2];
  z[2 * j] = x.re / scale;
  z[2 * j + 1] = x.im / scale;
}

// HE Add (Sec. III-B): c3 = c1 + c2 limb by limb, [2][level][N].
__global__ __launch_bounds__(THREADS) void k_he_add(const u64* a, const u64* b, u64* c, const ModInfo* mods,
                                                    u32 level, u32 log_n) {
  const u64 N = 1ull << log_n;
  const u64 e = (u64)blockIdx.x * THREADS + threadIdx.x;
  if (e >= 2ull * level * N) return;
  const u32 i = (u32)((e >> log_n) % level);
  const u64 q = mods[i].q;
  c[e] = addmod(a[e], b[e], q);
}

}  // namespace enc
}  // namespace he
