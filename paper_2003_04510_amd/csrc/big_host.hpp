// Host side and C ABI of the paper's non-RNS HE Mul (Sec. III, Fig. 2; see
// bigint.hpp for the kernels).  Included by he_lib.hip after its own C ABI:
// it reuses that file's NTT dispatch (ntt_launch), timing and table helpers.
#include "bigint.hpp"

// Big-integer HE Mul context: the NTT tables of the region primes (an
// NTT-only he_ctx: region 1 uses the first np1 primes, region 2 all np2) and
// the CRT / iCRT tables.
struct he_big_ctx {
  he_ctx* ntt = nullptr;
  u32 log_n = 0, logQ = 0, np1 = 0, np2 = 0, W = 0, W2 = 0, C1 = 0, C2 = 0, Pc1 = 0, Pc2 = 0;
  u32 kb_ct = 0, kb_evk = 0;       // CRT k-blocks (32 bytes) of a ciphertext / key coefficient
  u64 N = 0;
  int device = 0;
  std::vector<u64> primes;
  uint8_t* blob = nullptr;
  const u64* crtB = nullptr;       // [4 kb_evk][crt_cols]: CRT matrix (balanced digits)
  u32 crt_cols = 0;                // 32 ceil(np2 / 4): whole four-prime steps
  const u64 *adj_ct = nullptr, *adj_evk = nullptr;  // [np2]: offset corrections of the CRT
  const u64* iscale1 = nullptr;    // [np1][2]: N^-1 [(M1/p_i)^-1]_{p_i}, Shoup pairs
  const u64* iscale2 = nullptr;    // [np2][2]
  const double* pinv = nullptr;    // [np2]
  const u64 *B1 = nullptr, *B2 = nullptr;            // [64][Pc]: iCRT Toeplitz fragments
  const long long *CW1 = nullptr, *CW2 = nullptr;    // [C]: iCRT offset corrections per word column
  const u32 *negM1 = nullptr, *negM2 = nullptr;      // [C]: words of -M mod 2^(32 C)
};

namespace {

// An NTT-only context over `mods` (moduli, twiddles, identity limb map).
he_status ntt_ctx_create(u32 log_n, const std::vector<u64>& mods, int device, he_ctx** out) {
  const u64 N = 1ull << log_n;
  std::unique_ptr<he_ctx, void (*)(he_ctx*)> c(new he_ctx, he_ctx_destroy);
  c->log_n = log_n; c->N = N; c->device = device;
  c->L = (u32)mods.size(); c->K = 0; c->dnum = 1; c->alpha = c->L;
  c->mod = mods;
  const u32 nm = (u32)mods.size();
  Blob B;
  std::vector<ModInfo> mi(nm);
  for (u32 i = 0; i < nm; ++i) mi[i] = make_modinfo(mods[i], N);
  const size_t o_mods = B.add(mi);
  std::vector<Tw2> tw(nm * N), itw(nm * N);
  std::vector<u32> idx(nm);
  for (u32 i = 0; i < nm; ++i) {
    idx[i] = i;
    const u64 m = mods[i];
    const u64 psi = min_root_2n(m, log_n), psii = invmod(psi, m);
    std::vector<u64> pw(N), ipw(N), bw(N), ibw(N);
    pw[0] = ipw[0] = 1;
    for (u64 k = 1; k < N; ++k) { pw[k] = mulmod(pw[k - 1], psi, m); ipw[k] = mulmod(ipw[k - 1], psii, m); }
    for (u64 k = 0; k < N; ++k) {
      const unsigned e = bitrev((unsigned)k, log_n);
      bw[k] = pw[e];
      ibw[k] = ipw[e];
    }
    tw_fill(tw.data() + i * N, bw, m, N);
    tw_fill(itw.data() + i * N, ibw, m, N);
  }
  const size_t o_tw = B.add(tw), o_itw = B.add(itw), o_iota = B.add(idx);
  HIP_TRY(hipSetDevice(device));
  HIP_TRY(hipMalloc(&c->blob, B.bytes.size()));
  HIP_TRY(hipMemcpy(c->blob, B.bytes.data(), B.bytes.size(), hipMemcpyHostToDevice));
  c->mods = (const ModInfo*)(c->blob + o_mods);
  c->tw = (const Tw2*)(c->blob + o_tw);
  c->itw = (const Tw2*)(c->blob + o_itw);
  c->iota = (const u32*)(c->blob + o_iota);
  *out = c.release();
  return HE_OK;
}

// Little-endian 32-bit word vectors for the iCRT tables.
typedef std::vector<uint32_t> Words;
void words_mul(Words& a, u64 m) {  // a *= m
  u128 cy = 0;
  for (auto& w : a) {
    const u128 t = (u128)w * m + cy;
    w = (uint32_t)t;
    cy = t >> 32;
  }
  while (cy) {
    a.push_back((uint32_t)cy);
    cy >>= 32;
  }
}
Words words_trunc(const Words& a, u32 n) {
  Words r(n, 0);
  for (u32 i = 0; i < n && i < a.size(); ++i) r[i] = a[i];
  return r;
}
Words words_neg(const Words& a) {  // -a mod 2^(32 |a|)
  Words r(a.size());
  u64 cy = 1;
  for (size_t i = 0; i < a.size(); ++i) {
    const u64 t = (u64)(uint32_t)~a[i] + cy;
    r[i] = (uint32_t)t;
    cy = t >> 32;
  }
  return r;
}
// Balanced base-256 digits in [-128, 127] of the little-endian bytes
// `bytes` (the final carry, of weight 256^n, is dropped: callers need the
// value modulo 256^n or know it to be zero).
std::vector<int> balanced(const std::vector<uint8_t>& bytes) {
  std::vector<int> d(bytes.size());
  int cy = 0;
  for (size_t i = 0; i < bytes.size(); ++i) {
    int v = bytes[i] + cy;
    cy = 0;
    if (v >= 128) {
      v -= 256;
      cy = 1;
    }
    d[i] = v;
  }
  return d;
}
u64 pack8(const int* d) {  // 8 signed digits -> bytes of a word
  u64 w = 0;
  for (int j = 0; j < 8; ++j) w |= (u64)(uint8_t)(int8_t)d[j] << (8 * j);
  return w;
}
double log2_sum(const std::vector<u64>& p, u32 n) {
  double s = 0;
  for (u32 i = 0; i < n; ++i) s += std::log2((double)p[i]);
  return s;
}

constexpr u32 MF_ROWS = big::MF_THREADS / 4;  // coefficients per matrix-core workgroup

void icrt_launch(const big::IcrtArgs& a, u32 njobs, hipStream_t st) {
  const u32 blocks = (u32)((1ull << a.log_n) / MF_ROWS);
  hipLaunchKernelGGL(big::k_big_icrt, dim3(blocks, njobs), dim3(big::MF_THREADS), 0, st, a);
}
void crt_launch(const big::CrtArgs& a, u32 njobs, hipStream_t st) {
  const u32 blocks = (u32)((1ull << a.log_n) / MF_ROWS);
  hipLaunchKernelGGL(big::k_big_crt, dim3(blocks, njobs), dim3(big::MF_THREADS), 0, st, a);
}

size_t big_ws_limbs(const he_big_ctx* b) { return 4ull * b->np1 + 3ull * b->W + 2ull * b->np2 + 2ull * b->W; }

}  // namespace

extern "C" {

he_status he_big_ctx_create(uint32_t log_n, uint32_t logQ, int device, he_big_ctx** out) {
  if (!out) return fail(HE_EINVAL, "he_big_ctx_create: null pointer");
  *out = nullptr;
  if (log_n < 12 || log_n > 17) return fail(HE_EUNSUPPORTED, "log_n must be in [12, 17]");
  if (logQ < 64 || logQ > 64 * big::WMAX) return fail(HE_EUNSUPPORTED, "log Q must be in [64, %d]", 64 * big::WMAX);
  std::unique_ptr<he_big_ctx> b(new he_big_ctx);
  b->log_n = log_n; b->logQ = logQ; b->N = 1ull << log_n; b->device = device;
  b->W = (logQ + 63) / 64;
  b->W2 = (2 * logQ + 63) / 64;
  // 60-bit primes, 1 mod 2N.  Region 1 holds products of two log Q-bit
  // polynomials, region 2 products of a log Q-bit one with the evaluation
  // key (2 log Q bits): |X| < N 2^bits, so M > 2^(bits + log N + 3) keeps
  // the centred value within M/4.
  // (Region 1's Karatsuba sums are not reduced mod q: two more bits.)
  const double need1 = 2.0 * logQ + log_n + 5, need2 = 3.0 * logQ + log_n + 3;
  std::vector<u64> pr(64);
  if (!gen_primes(log_n, 60, 64, nullptr, 0, pr.data())) return fail(HE_EINVAL, "he_big_ctx_create: primes");
  u32 np1 = 1, np2 = 1;
  while (log2_sum(pr, np1) <= need1) ++np1;
  while (np2 <= 64 && log2_sum(pr, np2) <= need2) ++np2;
  if (np2 > 64) return fail(HE_EUNSUPPORTED, "log Q %u needs more than 64 primes", logQ);
  pr.resize(np2);
  b->primes = pr; b->np1 = np1; b->np2 = np2;
  b->C1 = (logQ + 31) / 32 + 1;
  b->C2 = (2 * logQ + 31) / 32 + 1;
  b->Pc1 = 16 * ((b->C1 + 3) / 4);
  b->Pc2 = 16 * ((b->C2 + 3) / 4);
  b->kb_ct = (b->W + 3) / 4;
  b->kb_evk = (b->W2 + 3) / 4;
  if (np2 > 64 || b->kb_evk > (u32)big::CRT_KBMAX) return fail(HE_EUNSUPPORTED, "log Q %u too large", logQ);
  he_status r = ntt_ctx_create(log_n, pr, device, &b->ntt);
  if (r != HE_OK) return r;
  const u64 N = b->N;
  Blob B;
  // CRT matrix: column 8i + b, k = byte h: digit b of c_{i,h} = [2^(8h)]_{p_i}
  // (balanced), stored word-major [kw][column] so 16 lanes read 128
  // contiguous bytes; whole steps of four primes (zero columns past np2).
  const u32 KW = 4 * b->kb_evk, KP = 8 * KW;
  b->crt_cols = 32 * ((np2 + 3) / 4);
  std::vector<u64> crtB((size_t)KW * b->crt_cols, 0);
  std::vector<u64> adj_ct(np2), adj_evk(np2);
  for (u32 i = 0; i < np2; ++i) {
    const u64 p = pr[i];
    std::vector<std::vector<int>> dig(KP);
    u64 sum_ct = 0, sum_evk = 0;  // sum_h c_{i,h} mod p over the k-range of each use
    for (u32 h = 0; h < KP; ++h) {
      const u64 c = powmod(2, 8ull * h, p);
      std::vector<uint8_t> by(8);
      for (int t = 0; t < 8; ++t) by[t] = (uint8_t)(c >> (8 * t));
      dig[h] = balanced(by);  // c < 2^60: eight digits, no final carry
      if (h < 32 * b->kb_ct) sum_ct = addmod(sum_ct, c, p);
      sum_evk = addmod(sum_evk, c, p);
    }
    for (u32 bd = 0; bd < 8; ++bd)
      for (u32 kw = 0; kw < KW; ++kw) {
        int d8[8];
        for (int j = 0; j < 8; ++j) d8[j] = dig[8 * kw + j][bd];
        crtB[(size_t)kw * b->crt_cols + 8 * i + bd] = pack8(d8);
      }
    const u64 t80 = powmod(2, 80, p);
    adj_ct[i] = submod(mulmod(128 % p, sum_ct, p), t80, p);
    adj_evk[i] = submod(mulmod(128 % p, sum_evk, p), t80, p);
  }
  const size_t o_crtB = B.add(crtB), o_adj_ct = B.add(adj_ct), o_adj_evk = B.add(adj_evk);
  std::vector<double> pinv(np2);
  for (u32 i = 0; i < np2; ++i) pinv[i] = 1.0 / (double)pr[i];
  const size_t o_pinv = B.add(pinv);
  // iCRT tables of a region over the first np primes, C word columns:
  // fragments B[i][P] (byte j = digit P - j of (M/p_i) mod 2^(32 C)),
  // offset corrections per word column, -M mod 2^(32 C), inverse NTT scales.
  auto region = [&](u32 np, u32 C, u32 Pc, size_t& o_sc, size_t& o_B, size_t& o_cw, size_t& o_nM) {
    std::vector<u64> sc(2 * np);
    std::vector<u64> Bt((size_t)64 * Pc, 0);
    std::vector<long long> colsum(Pc, 0), cw(C, 0);
    Words M{1};
    for (u32 i = 0; i < np; ++i) words_mul(M, pr[i]);
    for (u32 i = 0; i < np; ++i) {
      Words Mi{1};
      u64 mi = 1;  // (M / p_i) mod p_i
      for (u32 j = 0; j < np; ++j)
        if (j != i) {
          words_mul(Mi, pr[j]);
          mi = mulmod(mi, pr[j] % pr[i], pr[i]);
        }
      const u64 v = mulmod(invmod(N % pr[i], pr[i]), invmod(mi, pr[i]), pr[i]);
      sc[2 * i] = v;
      sc[2 * i + 1] = shoup(v, pr[i]);
      const Words t = words_trunc(Mi, C);
      std::vector<uint8_t> by(4 * C);
      for (u32 q = 0; q < 4 * C; ++q) by[q] = (uint8_t)(t[q / 4] >> (8 * (q % 4)));
      const std::vector<int> d = balanced(by);  // mod 2^(32 C): the final carry drops out
      for (u32 P = 0; P < Pc; ++P) {
        int d8[8];
        for (int j = 0; j < 8; ++j) {
          const int q = (int)P - j;
          d8[j] = (q >= 0 && q < (int)(4 * C)) ? d[q] : 0;
          colsum[P] += d8[j];
        }
        Bt[(size_t)i * Pc + P] = pack8(d8);
      }
    }
    for (u32 m = 0; m < C; ++m)
      for (u32 bb = 0; bb < 4; ++bb) cw[m] += 128ll * colsum[4 * m + bb] * (1ll << (8 * bb));
    const Words nM = words_neg(words_trunc(M, C));
    o_sc = B.add(sc); o_B = B.add(Bt); o_cw = B.add(cw); o_nM = B.add(nM);
  };
  size_t o_s1, o_B1, o_c1, o_n1, o_s2, o_B2, o_c2, o_n2;
  region(np1, b->C1, b->Pc1, o_s1, o_B1, o_c1, o_n1);
  region(np2, b->C2, b->Pc2, o_s2, o_B2, o_c2, o_n2);
  HIP_TRY(hipSetDevice(device));
  HIP_TRY(hipMalloc(&b->blob, B.bytes.size()));
  {
    hipError_t e = hipMemcpy(b->blob, B.bytes.data(), B.bytes.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      he_big_ctx_destroy(b.release());
      return fail(HE_EDEVICE, "table upload failed: %s", hipGetErrorString(e));
    }
  }
  uint8_t* d = b->blob;
  b->crtB = (const u64*)(d + o_crtB);
  b->adj_ct = (const u64*)(d + o_adj_ct); b->adj_evk = (const u64*)(d + o_adj_evk);
  b->pinv = (const double*)(d + o_pinv);
  b->iscale1 = (const u64*)(d + o_s1); b->B1 = (const u64*)(d + o_B1);
  b->CW1 = (const long long*)(d + o_c1); b->negM1 = (const u32*)(d + o_n1);
  b->iscale2 = (const u64*)(d + o_s2); b->B2 = (const u64*)(d + o_B2);
  b->CW2 = (const long long*)(d + o_c2); b->negM2 = (const u32*)(d + o_n2);
  *out = b.release();
  return HE_OK;
}

void he_big_ctx_destroy(he_big_ctx* b) {
  if (!b) return;
  if (b->blob) {
    (void)hipSetDevice(b->device);
    (void)hipFree(b->blob);
  }
  he_ctx_destroy(b->ntt);
  delete b;
}

he_status he_big_info(const he_big_ctx* b, uint32_t* np1, uint32_t* np2, uint32_t* words, uint64_t* primes) {
  if (!b) return fail(HE_EINVAL, "he_big_info: null context");
  if (np1) *np1 = b->np1;
  if (np2) *np2 = b->np2;
  if (words) *words = b->W;
  if (primes) memcpy(primes, b->primes.data(), b->primes.size() * sizeof(u64));
  return HE_OK;
}

size_t he_big_ct_bytes(const he_big_ctx* b) { return b ? 2ull * b->W * b->N * 8 : 0; }
size_t he_big_evk_bytes(const he_big_ctx* b) { return b ? 2ull * b->W2 * b->N * 8 : 0; }
size_t he_big_evk_ntt_bytes(const he_big_ctx* b) { return b ? 2ull * b->np2 * b->N * 8 : 0; }
size_t he_big_workspace_bytes(const he_big_ctx* b) { return b ? big_ws_limbs(b) * b->N * 8 : 0; }

he_status he_big_evk_prepare(he_big_ctx* b, const uint64_t* d_evk, uint64_t* d_evk_ntt, he_stream stream) {
  if (!b || !d_evk || !d_evk_ntt) return fail(HE_EINVAL, "he_big_evk_prepare: null pointer");
  HIP_TRY(hipSetDevice(b->device));
  hipStream_t st = (hipStream_t)stream;
  const u64 N = b->N;
  big::CrtArgs a{};
  for (int u = 0; u < 2; ++u) {
    a.src[u] = d_evk + (u64)u * b->W2 * N;
    a.dst[u] = d_evk_ntt + (u64)u * b->np2 * N;
  }
  a.mods = b->ntt->mods; a.B = b->crtB; a.adj = b->adj_evk; a.np = b->np2; a.W = b->W2;
  a.kb = b->kb_evk; a.ncols = b->crt_cols; a.log_n = b->log_n;
  crt_launch(a, 2, st);
  ntt_launch(b->ntt, true, d_evk_ntt, d_evk_ntt, N, N, b->np2 * N, b->np2 * N, b->ntt->iota, nullptr, b->np2, 2,
             st);
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

he_status he_big_mul(he_big_ctx* b, uint32_t logq, const uint64_t* d_ct1, const uint64_t* d_ct2,
                     const uint64_t* d_evk_ntt, uint64_t* d_out, uint32_t logp, void* ws, size_t ws_bytes,
                     he_stream stream) {
  if (!b || !d_ct1 || !d_ct2 || !d_evk_ntt || !d_out || !ws) return fail(HE_EINVAL, "he_big_mul: null pointer");
  if (logq < 1 || logq > b->logQ) return fail(HE_ELEVEL, "he_big_mul: log q %u not in [1, %u]", logq, b->logQ);
  if (logp >= logq || logp > 63) return fail(HE_EINVAL, "he_big_mul: log p %u must be below log q and 64", logp);
  if (ws_bytes < he_big_workspace_bytes(b)) return fail(HE_ENOMEM, "he_big_mul: workspace too small");
  const u64 N = b->N, W = b->W, ct = 2 * W * N * 8;
  auto overlaps = [](const void* x, size_t nx, const void* y, size_t ny) {
    return (const uint8_t*)x < (const uint8_t*)y + ny && (const uint8_t*)y < (const uint8_t*)x + nx;
  };
  if (overlaps(d_out, ct, d_ct1, ct) || overlaps(d_out, ct, d_ct2, ct))
    return fail(HE_EINVAL, "he_big_mul: output aliases an input");
  HIP_TRY(hipSetDevice(b->device));
  hipStream_t st = (hipStream_t)stream;
  he_ctx* nc = b->ntt;
  const u32 np1 = b->np1, np2 = b->np2;
  u64* R1 = (u64*)ws;                  // [4][np1][N]: ax1, ax2, bx1, bx2 -> axbx, axax, bxbx
  u64* B1 = R1 + 4ull * np1 * N;       // [3][W][N]: axbx, axax, bxbx
  u64* R2 = B1 + 3ull * W * N;         // [2][np2][N]
  u64* KS = R2 + 2ull * np2 * N;       // [2][W][N]: ks_b, ks_a
  const u64 L1 = (u64)np1 * N, L2 = (u64)np2 * N, WN = W * N;
  const u64 *bx1 = d_ct1, *ax1 = d_ct1 + WN, *bx2 = d_ct2, *ax2 = d_ct2 + WN;
  const double cN = (double)N;
  auto crt = [&](u32 njobs, const big::CrtArgs& a) {
    timed(nc, "big_crt", cN * njobs * a.np * 8 * 32 * a.kb, cN * njobs * (W + (u64)a.np) * 8, st,
          [&] { crt_launch(a, njobs, st); });
  };
  auto icrt = [&](u32 njobs, const big::IcrtArgs& a) {
    timed(nc, "big_icrt", cN * njobs * 32 * a.kb * 16 * ((a.C + 3) / 4), cN * njobs * ((u64)a.np + W) * 8, st,
          [&] { icrt_launch(a, njobs, st); });
  };
  // region 1: CRT of ax1, ax2, bx1, bx2
  {
    big::CrtArgs a{};
    const u64* srcs[4] = {ax1, ax2, bx1, bx2};
    for (int u = 0; u < 4; ++u) {
      a.src[u] = srcs[u];
      a.dst[u] = R1 + u * L1;
    }
    a.mods = nc->mods; a.B = b->crtB; a.adj = b->adj_ct; a.np = np1; a.W = (u32)W; a.kb = b->kb_ct;
    a.ncols = b->crt_cols; a.log_n = b->log_n;
    crt(4, a);
  }
  ntt_launch(nc, true, R1, R1, N, N, L1, L1, nc->iota, nullptr, np1, 4, st);
  timed(nc, "big_pointwise", cN * np1 * 3, cN * np1 * 7 * 8, st, [&] {
    hipLaunchKernelGGL(big::k_big_mul_r1, dim3((u32)(L1 / 256)), dim3(256), 0, st, R1, nc->mods, np1, b->log_n);
  });
  ntt_launch(nc, false, R1, R1, N, N, L1, L1, nc->iota, b->iscale1, np1, 3, st);
  {
    big::IcrtArgs a{};
    a.src = R1; a.dst = B1; a.pinv = b->pinv; a.B = b->B1; a.CW = b->CW1; a.negM = b->negM1;
    a.np = np1; a.kb = (np1 + 3) / 4; a.Pc = b->Pc1;
    a.shift = 0; a.round = 0; a.outbits = logq; a.W = (u32)W; a.log_n = b->log_n;
    a.C = std::min(b->C1, (logq + 31) / 32 + 1);
    icrt(3, a);
  }
  // region 2: axax times the evaluation key, shifted right by log Q
  {
    big::CrtArgs a{};
    a.src[0] = B1 + WN;
    a.dst[0] = R2;
    a.mods = nc->mods; a.B = b->crtB; a.adj = b->adj_ct; a.np = np2; a.W = (u32)W; a.kb = b->kb_ct;
    a.ncols = b->crt_cols; a.log_n = b->log_n;
    crt(1, a);
  }
  ntt_launch(nc, true, R2, R2, N, N, 0, 0, nc->iota, nullptr, np2, 1, st);
  {
    big::MulArgs a{};
    // the ax product first: the bx product overwrites the shared operand
    a.x[0] = R2; a.y[0] = d_evk_ntt + L2; a.out[0] = R2 + L2;
    a.x[1] = R2; a.y[1] = d_evk_ntt; a.out[1] = R2;
    a.mods = nc->mods; a.np = np2; a.nk = 2; a.log_n = b->log_n;
    timed(nc, "big_pointwise", cN * np2 * 2, cN * np2 * 5 * 8, st, [&] {
      hipLaunchKernelGGL(big::k_big_mul, dim3((u32)(L2 / 256)), dim3(256), 0, st, a);
    });
  }
  ntt_launch(nc, false, R2, R2, N, N, L2, L2, nc->iota, b->iscale2, np2, 2, st);
  {
    big::IcrtArgs a{};
    a.src = R2; a.dst = KS; a.pinv = b->pinv; a.B = b->B2; a.CW = b->CW2; a.negM = b->negM2;
    a.np = np2; a.kb = (np2 + 3) / 4; a.Pc = b->Pc2;
    a.shift = b->logQ; a.round = 1; a.outbits = logq; a.W = (u32)W; a.log_n = b->log_n;
    a.C = std::min(b->C2, (b->logQ + logq + 31) / 32 + 1);
    icrt(2, a);
  }
  {
    big::FinArgs a{};
    a.ks = KS; a.r1 = B1; a.out = d_out; a.W = (u32)W; a.logq = logq; a.logp = logp; a.log_n = b->log_n;
    timed(nc, "big_finish", cN * 2 * W, cN * (5 + 2) * W * 8, st, [&] {
      hipLaunchKernelGGL(big::k_big_finish, dim3((u32)(N / big::FIN_THREADS), 2), dim3(big::FIN_THREADS), 0, st, a);
    });
  }
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

he_status he_big_timing_enable(he_big_ctx* b, int enable) {
  if (!b) return fail(HE_EINVAL, "he_big_timing_enable: null context");
  return he_timing_enable(b->ntt, enable, nullptr);
}

he_status he_big_timing_read(he_big_ctx* b, he_kernel_stat* out, uint32_t max, uint32_t* n) {
  if (!b) return fail(HE_EINVAL, "he_big_timing_read: null context");
  return he_timing_read(b->ntt, out, max, n);
}

}  // extern "C"
