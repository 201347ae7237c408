// C-ABI library: context (moduli, twiddle and base-conversion tables on the
// device), key generation, encryption, decryption, HE Mul and rescale.
// All device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/he_mi355x.h"
#include "host_math.hpp"
#include "ntt.hpp"
#include "fused.hpp"
#include "launch.hpp"
#include "rns_kernels.hpp"
#include "ubench.hpp"

using namespace he;

namespace {

thread_local std::string g_err;

// Scratch of he_mul_noalloc: one array per GPU, alive until the process
// ends.  In host code `scratch` is only a handle for the symbol lookup; the
// device address of each GPU's copy is taken once per device (with that
// device current) and kept in g_scratch.
static __device__ __align__(256) uint64_t scratch[HE_NOALLOC_SCRATCH_BYTES / 8];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[MAX_DEVICES] = {};

he_status fail(he_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

}  // namespace

// Error message of a failing call, for the other translation units of the
// library (the serving loop).
void he_set_last_error(const char* msg) { g_err = msg ? msg : ""; }

namespace {

#define HIP_TRY(x)                                                                   \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess)                                                            \
      return fail(HE_EDEVICE, "%s failed: %s (%s:%d)", #x, hipGetErrorString(e_),    \
                  __FILE__, __LINE__);                                               \
  } while (0)

// Host-side builder for one device blob of constant tables.  With `sizing`
// set it only accounts for the layout (offsets and total size), so the size
// query needs neither the tables nor their memory.
struct Blob {
  bool sizing = false;
  size_t size = 0;
  std::vector<uint8_t> bytes;
  size_t add(const void* p, size_t n) {
    const size_t off = (size + 255) & ~size_t(255);
    size = off + n;
    if (!sizing) {
      bytes.resize(size);
      if (n && p) memcpy(bytes.data() + off, p, n);
    }
    return off;
  }
  template <class T>
  size_t add(const std::vector<T>& v) { return add(v.data(), v.size() * sizeof(T)); }
};

// One base-conversion job as planned on the host: sources src_off .. +ns,
// targets dst_off .. +nt, constants C[s][t] at c_off, target moduli at m_off.
struct ConvJob {
  u32 src_off, ns, dst_off, nt, c_off, m_off;
};

struct LevelPlan {
  u32 beta = 0, dt_limbs = 0;
  size_t o_mu_c = 0, o_md_c = 0, o_y_mod = 0, o_y_scale = 0, o_s_mod = 0, o_s_scale = 0;
  const u32* mu_c = nullptr;  // mod-up conversion records [dt_limbs] (see conv_rec_words)
  const u32* md_c = nullptr;  // mod-down conversion records [level]
  const u32* y_mod = nullptr;         // INTT list of d2 (+ d0, d1 of the last limb): [level + 2]
  const u64* y_scale = nullptr;
  const u32* s_mod = nullptr;         // INTT list of the special limbs (+ limb level-1): [K + 1]
  const u64* s_scale = nullptr;
  size_t o_mu_jobs = 0, o_md_jobs = 0;
  const ConvJobDev* mu_jobs = nullptr;  // [beta]
  const ConvJobDev* md_jobs = nullptr;  // [1]
  u32 lo[MAX_DIGITS] = {}, cnt[MAX_DIGITS] = {}, dt_first[MAX_DIGITS] = {};
  size_t o_modup_scale = 0, o_dt_mod = 0, o_emod = 0, o_qlinv = 0, o_qlmod = 0, o_dtg_limb = 0, o_dtg_first = 0;
  u32 dtg_count = 0;
  // resolved device pointers
  const u64* modup_scale = nullptr;
  const u32* dt_mod = nullptr;
  const u32* emod = nullptr;
  const u64* qlinv = nullptr;
  const u64* qlmod = nullptr;
  size_t o_plan = 0;
  const PlanDev* plan = nullptr;  // device copy of this level's plan
  u64 pinv_l = 0;                 // [P^-1]_{q_{level-1}}
};

}  // namespace

struct he_ctx {
  u32 log_n = 0, L = 0, K = 0, dnum = 0, alpha = 0;
  u64 N = 0;
  int device = 0;
  std::vector<u64> mod;        // [L+K]
  std::vector<u64> pmod_host;  // [P]_{m} for every modulus m
  bool w32 = false;            // residues stored as 32-bit words (every prime below 2^31)
  uint8_t* blob = nullptr;     // device constant tables
  size_t blob_bytes = 0;
  bool owns_blob = true;       // false: caller-provided table memory
  // device pointers into blob
  const ModInfo* mods = nullptr;
  const Tw2 *tw = nullptr, *itw = nullptr;
  const double *gtw = nullptr, *igtw = nullptr;  // factored blocks-pass twiddles (FP64 moduli)
  u32 gstride = 0;
  const u32* iota = nullptr;
  const u64* spec_scale = nullptr;  // [K] pairs: N^-1 [(P/p_k)^-1]_{p_k}
  const u64* pinv = nullptr;        // [L] pairs: [P^-1]_{q_i}
  const u64* pmod = nullptr;        // [L+K]: [P]_m
  std::vector<LevelPlan> lv;        // index = level (1..L)
  // optional per-kernel timing (diagnostics)
  bool timing = false;
  std::string timing_only;          // empty = every kernel
  struct TRec {
    const char* name;
    hipEvent_t a, b;
    double ops, bytes;
  };
  std::vector<TRec> trecs;
  std::vector<hipEvent_t> tpool;
};

namespace {

size_t ceil_div(size_t a, size_t b) { return (a + b - 1) / b; }

// Bytes of one stored residue (a 64-bit or, for 32-bit-word contexts, a
// 32-bit word).
inline u64 word_bytes(const he_ctx* c) { return c->w32 ? 4 : 8; }

// Entry points that move 64-bit words only.
he_status need_w64(const he_ctx* c, const char* fn) {
  if (c && c->w32) return fail(HE_EUNSUPPORTED, "%s: not available for 32-bit-word contexts (use he_mul32)", fn);
  return HE_OK;
}

hipEvent_t pool_event(he_ctx* c) {
  if (!c->tpool.empty()) {
    hipEvent_t e = c->tpool.back();
    c->tpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run `launch` (which enqueues one kernel on st); when timing is on for
// `name`, bracket it with events and record its algorithmic work.
template <class F>
void timed(const he_ctx* cc, const char* name, double ops, double bytes, hipStream_t st, F&& launch) {
  he_ctx* c = const_cast<he_ctx*>(cc);
  const bool on = c->timing && (c->timing_only.empty() || c->timing_only == name);
  hipEvent_t a = nullptr, b = nullptr;
  if (on) {
    a = pool_event(c);
    b = pool_event(c);
    if (a && b) (void)hipEventRecord(a, st);
  }
  launch();
  if (on && a && b) {
    (void)hipEventRecord(b, st);
    c->trecs.push_back({name, a, b, ops, bytes});
  }
}

// ---------------------------------------------------------------- NTT dispatch
template <bool FWD, int LOGS>
void launch_cols(const he_ctx* c, const NttArgs& a, u32 nlimbs, u32 npolys, hipStream_t st) {
  using PG = PassGeo<LOGS>;
  const u32 ncols = 1u << (a.log_n - LOGS);
  const double units = (double)nlimbs * npolys;
  const double bfly = units * (double)(c->N / 2) * LOGS + (FWD ? 0.0 : units * (double)c->N);
  timed(c, FWD ? "ntt_cols" : "intt_cols", bfly, units * c->N * 16.0, st, [&] {
    hipLaunchKernelGGL((k_ntt_cols<FWD, LOGS>), dim3(ncols / PG::SUBS, nlimbs, npolys), dim3(PG::THREADS), 0, st,
                       a);
  });
}
template <bool FWD, int LOGS>
void launch_blocks(const he_ctx* c, const NttArgs& a, u32 nlimbs, u32 npolys, hipStream_t st) {
  using PG = PassGeo<LOGS>;
  const u32 nblk = 1u << (a.log_n - LOGS);
  const double units = (double)nlimbs * npolys;
  timed(c, FWD ? "ntt_blocks" : "intt_blocks", units * (double)(c->N / 2) * LOGS, units * c->N * 16.0, st, [&] {
    hipLaunchKernelGGL((k_ntt_blocks<FWD, LOGS>), dim3(nblk / PG::SUBS, nlimbs, npolys), dim3(PG::THREADS), 0,
                       st, a);
  });
}
template <bool FWD>
void cols_dispatch(const he_ctx* c, int logs, const NttArgs& a, u32 nl, u32 np, hipStream_t st) {
  switch (logs) {
    case 6: launch_cols<FWD, 6>(c, a, nl, np, st); break;
    case 7: launch_cols<FWD, 7>(c, a, nl, np, st); break;
    case 8: launch_cols<FWD, 8>(c, a, nl, np, st); break;
  }
}
template <bool FWD>
void blocks_dispatch(const he_ctx* c, int logs, const NttArgs& a, u32 nl, u32 np, hipStream_t st) {
  switch (logs) {
    case 6: launch_blocks<FWD, 6>(c, a, nl, np, st); break;
    case 7: launch_blocks<FWD, 7>(c, a, nl, np, st); break;
    case 8: launch_blocks<FWD, 8>(c, a, nl, np, st); break;
    case 9: launch_blocks<FWD, 9>(c, a, nl, np, st); break;
  }
}

// Transform nlimbs limbs (x npolys polynomials).  src may equal dst.
void ntt_launch(const he_ctx* c, bool fwd, const u64* src, u64* dst, u64 src_stride, u64 dst_stride,
                u64 src_z, u64 dst_z, const u32* limb_mod, const u64* scale, u32 nlimbs, u32 npolys,
                hipStream_t st) {
  if (!nlimbs || !npolys) return;
  const int n1 = (int)c->log_n / 2, n2 = (int)c->log_n - n1;
  NttArgs a{};
  a.limb_mod = limb_mod;
  a.mods = c->mods;
  a.log_n = c->log_n;
  a.scale = scale;
  if (fwd) {
    a.tw = c->tw;
    a.src = src; a.dst = dst; a.src_stride = src_stride; a.dst_stride = dst_stride;
    a.src_zstride = src_z; a.dst_zstride = dst_z;
    cols_dispatch<true>(c, n1, a, nlimbs, npolys, st);
    a.src = dst; a.src_stride = dst_stride; a.src_zstride = dst_z;
    blocks_dispatch<true>(c, n2, a, nlimbs, npolys, st);
  } else {
    a.tw = c->itw;
    a.src = src; a.dst = dst; a.src_stride = src_stride; a.dst_stride = dst_stride;
    a.src_zstride = src_z; a.dst_zstride = dst_z;
    blocks_dispatch<false>(c, n2, a, nlimbs, npolys, st);
    a.src = dst; a.src_stride = dst_stride; a.src_zstride = dst_z;
    cols_dispatch<false>(c, n1, a, nlimbs, npolys, st);
  }
}

dim3 ew_grid(u64 total) { return dim3((unsigned)ceil_div(total, EW_THREADS)); }

// ---------------------------------------------------------------- tables
// Twiddle table of modulus m (N entries of 16 bytes at t) in the form the
// kernels read for m: Shoup pairs, or for m < 2^50 the doubles W_k in the
// first half.
void tw_fill(Tw2* t, const std::vector<u64>& w, u64 m, u64 N, bool i32 = false) {
  if (i32) {  // 32-bit Shoup pairs: w | floor(w 2^32 / m) << 32, 8 bytes per index
    std::vector<u64> d(2 * N, 0);
    for (u64 k = 0; k < N; ++k) d[k] = w[k] | ((u64)(((u128)w[k] << 32) / m) << 32);
    memcpy(t, d.data(), N * sizeof(Tw2));
    return;
  }
  if (f64_mod(m)) {
    std::vector<double> d(2 * N, 0.0);
    for (u64 k = 0; k < N; ++k) d[k] = (double)w[k];  // exact: w < 2^50
    memcpy(t, d.data(), N * sizeof(Tw2));
    return;
  }
  for (u64 k = 0; k < N; ++k) t[k] = Tw2{w[k], shoup63(w[k], m)};
}

ModInfo make_modinfo(u64 q, u64 N) {
  ModInfo m{};
  m.q = q;
  m.b = bitlen(q);
  m.qinv = 1.0 / (double)q;
  m.mu = (u64)(((u128)1 << (2 * m.b)) / q);
  m.r64 = (u64)(((u128)1 << 64) % q);
  m.r64s = shoup(m.r64, q);
  m.one_s = (u64)(((u128)1 << 64) / q);
  m.ninv = invmod(N % q, q);
  m.ninvs = shoup(m.ninv, q);
  return m;
}

u64 prod_mod(const std::vector<u64>& ms, const std::vector<u32>& idx, u32 skip, u64 m) {
  u64 r = 1 % m;
  for (u32 i : idx)
    if (i != skip) r = mulmod(r, ms[i] % m, m);
  return r;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* he_status_str(he_status s) {
  switch (s) {
    case HE_OK: return "ok";
    case HE_EINVAL: return "invalid argument";
    case HE_ELEVEL: return "level out of range";
    case HE_ENOMEM: return "insufficient memory or workspace";
    case HE_EDEVICE: return "device error";
    case HE_EUNSUPPORTED: return "unsupported";
    case HE_EBUSY: return "busy";
  }
  return "unknown";
}

const char* he_last_error(void) { return g_err.c_str(); }

he_status he_timing_enable(he_ctx* c, int enable, const char* only) {
  if (!c) return fail(HE_EINVAL, "he_timing_enable: null context");
  c->timing = enable != 0;
  c->timing_only = only ? only : "";
  return HE_OK;
}

he_status he_timing_read(he_ctx* c, he_kernel_stat* out, uint32_t max, uint32_t* n) {
  if (!c || !n || (max && !out)) return fail(HE_EINVAL, "he_timing_read: null pointer");
  std::vector<he_kernel_stat> agg;
  for (auto& r : c->trecs) {
    float ms = 0;
    hipError_t e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return fail(HE_EDEVICE, "he_timing_read: %s (synchronize the stream first)",
                                     hipGetErrorString(e));
    size_t k = 0;
    while (k < agg.size() && strcmp(agg[k].name, r.name)) ++k;
    if (k == agg.size()) {
      he_kernel_stat z{};
      snprintf(z.name, sizeof z.name, "%s", r.name);
      agg.push_back(z);
    }
    agg[k].launches += 1;
    agg[k].ms += ms;
    agg[k].ops += r.ops;
    agg[k].bytes += r.bytes;
  }
  for (auto& r : c->trecs) {
    c->tpool.push_back(r.a);
    c->tpool.push_back(r.b);
  }
  c->trecs.clear();
  *n = (uint32_t)agg.size();
  for (uint32_t i = 0; i < agg.size() && i < max; ++i) out[i] = agg[i];
  return HE_OK;
}

he_status he_gen_primes(uint32_t log_n, uint32_t bits, uint32_t count, const uint64_t* exclude,
                        uint32_t nexclude, uint64_t* out) {
  if (!out || bits < 20 || bits > 61 || log_n < 1 || log_n > 20 || (nexclude && !exclude))
    return fail(HE_EINVAL, "he_gen_primes: bad arguments");
  if (!gen_primes(log_n, bits, count, exclude, nexclude, out))
    return fail(HE_EINVAL, "he_gen_primes: fewer than %u primes", count);
  return HE_OK;
}

}  // extern "C"

// Validates the parameters and lays out (sizing) or builds the context's
// constant tables.  sizing: only *table_bytes is produced.  Otherwise the
// tables go to d_tables (caller-owned, at least table_bytes long) or, when
// d_tables is null, to device memory the context allocates and owns.
static he_status ctx_make(uint32_t log_n, uint32_t L, uint32_t K, uint32_t dnum, const uint64_t* q,
                          const uint64_t* p, int device, bool sizing, void* d_tables, size_t tables_bytes,
                          size_t* table_bytes, he_ctx** out, bool w32 = false) {
  if ((!out && !sizing) || !q || !p) return fail(HE_EINVAL, "he_ctx_create: null pointer");
  if (out) *out = nullptr;
  if (log_n < 12 || log_n > 17) return fail(HE_EUNSUPPORTED, "log_n must be in [12, 17]");
  if (L < 1 || L > 64 || K < 1 || K > 32 || dnum < 1 || dnum > L || dnum > (u32)MAX_DIGITS)
    return fail(HE_EINVAL, "need 1 <= dnum <= min(L, %d), L <= 64, 1 <= K <= 32", MAX_DIGITS);
  const u64 N = 1ull << log_n;
  std::unique_ptr<he_ctx, void (*)(he_ctx*)> c(new he_ctx, he_ctx_destroy);  // frees device memory on errors
  c->log_n = log_n; c->L = L; c->K = K; c->dnum = dnum; c->N = N;
  c->w32 = w32;
  if (w32 && log_n > 16) return fail(HE_EUNSUPPORTED, "32-bit words: log_n must be in [12, 16]");
  c->alpha = (L + dnum - 1) / dnum;
  c->device = device;
  const u32 nm = L + K;
  c->mod.assign(q, q + L);
  c->mod.insert(c->mod.end(), p, p + K);
  for (u32 i = 0; i < nm; ++i) {
    const u64 m = c->mod[i];
    if (m >= (1ull << 60) || m < (1ull << 20) || (m - 1) % (2 * N) || !is_prime(m))
      return fail(HE_EINVAL, "modulus %u (%llu) is not a prime below 2^60 that is 1 mod 2N", i,
                  (unsigned long long)m);
    if (w32 && m >= (1ull << 31))
      return fail(HE_EINVAL, "32-bit words: modulus %u (%llu) is not below 2^31", i, (unsigned long long)m);
    for (u32 j = 0; j < i; ++j)
      if (c->mod[j] == m) return fail(HE_EINVAL, "moduli must be distinct");
  }
  if (c->alpha > 32 || K > 32)
    return fail(HE_EUNSUPPORTED, "digit size ceil(L/dnum) and K must be <= 32");
  if (L + K > CONV_GROUPS * CONV_MAXT)  // a conversion item stages at most CONV_MAXT target records
    return fail(HE_EUNSUPPORTED, "L + K must be <= %d", CONV_GROUPS * CONV_MAXT);
  // special primes must cover every digit: P > prod(digit)
  {
    long double lp = 0, ld = 0;
    for (u32 k = 0; k < K; ++k) lp += log2l((long double)p[k]);
    for (u32 j = 0; j < dnum; ++j) {
      ld = 0;
      for (u32 i = j * c->alpha; i < std::min(L, (j + 1) * c->alpha); ++i) ld += log2l((long double)q[i]);
      if (ld >= lp) return fail(HE_EINVAL, "special primes (%.1f bits) do not exceed digit %u (%.1f bits)",
                                (double)lp, j, (double)ld);
    }
  }
  std::vector<u32> all_idx(nm), pidx(K);
  for (u32 i = 0; i < nm; ++i) all_idx[i] = i;
  for (u32 k = 0; k < K; ++k) pidx[k] = L + k;

  Blob B;
  // moduli
  std::vector<ModInfo> mi(nm);
  // 32-bit words run their butterflies on the 32-bit integer multipliers
  // (I32A) when every prime is below 2^30 (measured 7% faster than the FP64
  // butterflies on the same words at N = 2^16, 40 primes)
  bool i32 = w32;
  for (u32 i = 0; i < nm; ++i) i32 = i32 && c->mod[i] < (1ull << 30);
  for (u32 i = 0; i < nm; ++i) {
    mi[i] = make_modinfo(c->mod[i], N);
    mi[i].arith = i32 ? ARITH_I32 : ARITH_AUTO;
  }
  B.sizing = sizing;
  const size_t o_mods = B.add(mi);
  // twiddles: TB_W[k] = psi^bitrev(k), TB_invW[k] = psi^-bitrev(k), + Shoup companions
  std::vector<Tw2> tw(sizing ? 0 : nm * N), itw(sizing ? 0 : nm * N);
  const u32 n1 = log_n / 2, n2 = log_n - n1;
  const size_t gst = ((size_t)1 << n2) + ((size_t)n2 << n1);  // words per modulus: gA, then gB
  std::vector<double> gt(sizing ? 0 : nm * gst, 0.0), igt(sizing ? 0 : nm * gst, 0.0);
  for (u32 i = 0; i < nm && !sizing; ++i) {
    const u64 m = c->mod[i];
    const u64 psi = min_root_2n(m, log_n), psii = invmod(psi, m);
    std::vector<u64> pw(N), ipw(N);
    pw[0] = ipw[0] = 1;
    for (u64 k = 1; k < N; ++k) { pw[k] = mulmod(pw[k - 1], psi, m); ipw[k] = mulmod(ipw[k - 1], psii, m); }
    std::vector<u64> bw(N), ibw(N);
    for (u64 k = 0; k < N; ++k) {
      const unsigned e = bitrev((unsigned)k, log_n);
      bw[k] = pw[e];
      ibw[k] = ipw[e];
    }
    tw_fill(tw.data() + i * N, bw, m, N, i32);
    tw_fill(itw.data() + i * N, ibw, m, N, i32);
    // Blocks passes (n1 = log_n / 2 cols stages done, sub-transforms of
    // 2^n2 points) at stage s < n2, group t < 2^s of row block blk read
    // TB_W[2^(n1+s) + blk 2^s + t] = psi^(brv_s(t) 2^(log_n-s)) *
    // psi^((2 brv_n1(blk) + 1) 2^(n2-1-s)): the first factor (gA, 2^n2 words)
    // is shared by all blocks, the second (gB, n2 words per block) by the
    // groups of a stage.  FP64 moduli form the product exactly instead of
    // reading the table entry.
    if (f64_mod(m)) {
      for (int dir = 0; dir < 2; ++dir) {
        const std::vector<u64>& p = dir ? ipw : pw;
        double* g = (dir ? igt.data() : gt.data()) + (size_t)i * gst;
        for (u32 s2 = 0; s2 < n2; ++s2)
          for (u32 t = 0; t < (1u << s2); ++t) g[(1u << s2) + t] = (double)p[(u64)bitrev(t, s2) << (log_n - s2)];
        for (u32 blk = 0; blk < (1u << n1); ++blk)
          for (u32 s2 = 0; s2 < n2; ++s2)
            g[(1u << n2) + blk * n2 + s2] = (double)p[(2ull * bitrev(blk, n1) + 1) << (n2 - 1 - s2)];
      }
    }
  }
  const size_t o_tw = B.add(tw.data(), nm * N * sizeof(Tw2)), o_itw = B.add(itw.data(), nm * N * sizeof(Tw2));
  const size_t o_gt = B.add(gt.data(), nm * gst * sizeof(double)), o_igt = B.add(igt.data(), nm * gst * sizeof(double));
  const size_t o_iota = B.add(all_idx);
  // ModDown constants (level independent)
  std::vector<u64> spec_scale(2 * K), pinv(2 * L), pm(nm);
  for (u32 k = 0; k < K; ++k) {
    const u64 m = p[k];
    const u64 v = mulmod(invmod(N % m, m), invmod(prod_mod(c->mod, pidx, L + k, m), m), m);
    spec_scale[2 * k] = v;
    spec_scale[2 * k + 1] = shoup(v, m);
  }
  for (u32 i = 0; i < nm; ++i) pm[i] = prod_mod(c->mod, pidx, ~0u, c->mod[i]);
  for (u32 i = 0; i < L; ++i) {
    const u64 v = invmod(pm[i], q[i]);
    pinv[2 * i] = v;
    pinv[2 * i + 1] = shoup(v, q[i]);
  }
  c->pmod_host = pm;
  const size_t o_spec = B.add(spec_scale), o_pinv = B.add(pinv), o_pmod = B.add(pm);

  // per-level plans
  c->lv.resize(L + 1);
  for (u32 lvl = 1; lvl <= L; ++lvl) {
    LevelPlan& P = c->lv[lvl];
    P.beta = (lvl + c->alpha - 1) / c->alpha;
    const u32 ne = lvl + K;
    std::vector<u32> emod(ne);
    for (u32 e = 0; e < ne; ++e) emod[e] = e < lvl ? e : L + (e - lvl);
    std::vector<ConvJob> jobs(P.beta);
    std::vector<u64> consts, scale(2 * lvl);
    std::vector<u32> tmods, dt_mod;
    u32 dt_first = 0;
    for (u32 j = 0; j < P.beta; ++j) {
      const u32 lo = j * c->alpha, hi = std::min(lvl, (j + 1) * c->alpha);
      P.lo[j] = lo; P.cnt[j] = hi - lo; P.dt_first[j] = dt_first;
      std::vector<u32> dig;
      for (u32 i = lo; i < hi; ++i) dig.push_back(i);
      for (u32 i = lo; i < hi; ++i) {  // y_i scale: N^-1 [(Qt_j / q_i)^-1]_{q_i}
        const u64 m = q[i];
        const u64 v = mulmod(invmod(N % m, m), invmod(prod_mod(c->mod, dig, i, m), m), m);
        scale[2 * i] = v;
        scale[2 * i + 1] = shoup(v, m);
      }
      ConvJob& J = jobs[j];
      J.src_off = lo; J.ns = hi - lo; J.dst_off = dt_first; J.nt = ne - (hi - lo);
      J.c_off = (u32)consts.size(); J.m_off = (u32)tmods.size();
      std::vector<u32> tg;
      for (u32 e = 0; e < ne; ++e)
        if (!(e >= lo && e < hi)) tg.push_back(emod[e]);
      std::vector<u64> C((hi - lo) * tg.size());
      for (u32 s = 0; s < hi - lo; ++s)
        for (size_t t = 0; t < tg.size(); ++t) C[s * tg.size() + t] = prod_mod(c->mod, dig, lo + s, c->mod[tg[t]]);
      consts.insert(consts.end(), C.begin(), C.end());
      tmods.insert(tmods.end(), tg.begin(), tg.end());
      dt_mod.insert(dt_mod.end(), tg.begin(), tg.end());
      dt_first += (u32)tg.size();
    }
    P.dt_limbs = dt_first;
    // ModDown job: sources = K special limbs (after scaling), targets q_0..q_{lvl-1}
    ConvJob md{};
    md.src_off = lvl; md.ns = K; md.dst_off = 0; md.nt = lvl; md.c_off = 0; md.m_off = 0;
    std::vector<u64> mdc((size_t)K * lvl);
    for (u32 k = 0; k < K; ++k)
      for (u32 i = 0; i < lvl; ++i)  // [P/p_k]_{q_i} [P^-1]_{q_i}: the conversion yields z P^-1
        mdc[(size_t)k * lvl + i] = mulmod(prod_mod(c->mod, pidx, L + k, q[i]), pinv[2 * i], q[i]);
    // rescale constants
    std::vector<u64> qlinv(2 * (lvl > 1 ? lvl - 1 : 1), 0), qlmod(lvl > 1 ? lvl - 1 : 1, 0);
    for (u32 i = 0; i + 1 < lvl; ++i) {
      const u64 m = q[i], ql = q[lvl - 1] % m;
      qlmod[i] = ql;
      qlinv[2 * i] = invmod(ql, m);
      qlinv[2 * i + 1] = shoup(qlinv[2 * i], m);
    }
    // fused-kernel tables: one record per conversion target (its modulus's
    // reduction constants, then 30-bit split constants padded with zeros to
    // the kernel's source bound)
    {
      const auto record = [&](std::vector<u32>& out, u32 nsmax, u64 m, u64 extra, u32 ns, auto cst) {
        const ModInfo mi = make_modinfo(m, N);
        const u64 head[5] = {mi.q, mi.r64, mi.r64s, mi.one_s, extra};
        for (u64 h : head) {
          out.push_back((u32)h);
          out.push_back((u32)(h >> 32));
        }
        for (u32 s2 = 0; s2 < nsmax; ++s2) {
          const u64 cv = s2 < ns ? cst(s2) : 0;
          out.push_back((u32)(cv & M30));
          out.push_back((u32)(cv >> 30));
        }
      };
      const u32 mu_ns = (u32)conv_bucket(c->alpha), md_ns = (u32)conv_bucket(K);
      std::vector<u32> mc;
      for (u32 j = 0; j < P.beta; ++j) {
        const ConvJob& J = jobs[j];
        for (u32 t = 0; t < J.nt; ++t)
          record(mc, mu_ns, c->mod[tmods[J.m_off + t]], 0, J.ns,
                 [&](u32 s2) { return consts[J.c_off + (size_t)s2 * J.nt + t]; });
      }
      std::vector<u32> dc;
      for (u32 i = 0; i < lvl; ++i)
        record(dc, md_ns, q[i], i + 1 < lvl ? qlmod[i] : 0, K, [&](u32 k) { return mdc[(size_t)k * lvl + i]; });
      std::vector<u32> ymod(lvl + 2), smod(K + 1);
      std::vector<u64> ysc(2 * (lvl + 2)), ssc(2 * (K + 1));
      for (u32 i = 0; i < lvl; ++i) { ymod[i] = i; ysc[2 * i] = scale[2 * i]; ysc[2 * i + 1] = scale[2 * i + 1]; }
      const u64 ql = q[lvl - 1], nql = invmod(N % ql, ql);
      for (u32 k = 0; k < 2; ++k) { ymod[lvl + k] = lvl - 1; ysc[2 * (lvl + k)] = nql; ysc[2 * (lvl + k) + 1] = shoup(nql, ql); }
      for (u32 k = 0; k < K; ++k) { smod[k] = L + k; ssc[2 * k] = spec_scale[2 * k]; ssc[2 * k + 1] = spec_scale[2 * k + 1]; }
      smod[K] = lvl - 1; ssc[2 * K] = nql; ssc[2 * K + 1] = shoup(nql, ql);
      std::vector<ConvJobDev> mj(P.beta), dj(1);
      for (u32 j = 0; j < P.beta; ++j) mj[j] = {jobs[j].src_off, jobs[j].ns, jobs[j].dst_off, jobs[j].nt, jobs[j].dst_off, 0};
      dj[0] = {lvl, K, 0, lvl, 0, 0};
      P.o_mu_jobs = B.add(mj); P.o_md_jobs = B.add(dj);
      P.o_mu_c = B.add(mc); P.o_md_c = B.add(dc);
      P.o_y_mod = B.add(ymod); P.o_y_scale = B.add(ysc); P.o_s_mod = B.add(smod); P.o_s_scale = B.add(ssc);
    }
    P.o_modup_scale = B.add(scale); P.o_dt_mod = B.add(dt_mod); P.o_emod = B.add(emod);
    {
      // mod-up limbs grouped by modulus (stable), for the blocks pass's item order
      std::vector<u32> order(dt_mod.size()), first;
      for (u32 k = 0; k < order.size(); ++k) order[k] = k;
      std::stable_sort(order.begin(), order.end(), [&](u32 a, u32 b) { return dt_mod[a] < dt_mod[b]; });
      for (u32 k = 0; k < order.size(); ++k)
        if (k == 0 || dt_mod[order[k]] != dt_mod[order[k - 1]]) first.push_back(k);
      first.push_back((u32)order.size());
      P.dtg_count = (u32)first.size() - 1;
      P.o_dtg_limb = B.add(order);
      P.o_dtg_first = B.add(first);
    }
    P.o_qlinv = B.add(qlinv); P.o_qlmod = B.add(qlmod);
    {
      PlanDev placeholder{};
      P.o_plan = B.add(&placeholder, sizeof placeholder);
    }
    P.pinv_l = invmod(pm[lvl - 1], q[lvl - 1]);
    (void)md;
  }

  if (sizing) {
    *table_bytes = B.size;
    return HE_OK;
  }
  HIP_TRY(hipSetDevice(device));
  if (device < 0 || device >= MAX_DEVICES) return fail(HE_EINVAL, "he_ctx_create: device %d out of range", device);
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return fail(HE_EDEVICE, "he_ctx_create: scratch symbol lookup failed: %s", hipGetErrorString(e));
      g_scratch[device] = ptr;
    }
  }
  if (d_tables) {
    if (tables_bytes < B.size)
      return fail(HE_ENOMEM, "he_ctx_create: table memory of %zu bytes, need %zu", tables_bytes, B.size);
    c->blob = (uint8_t*)d_tables;
    c->owns_blob = false;
  } else {
    HIP_TRY(hipMalloc(&c->blob, B.size));
  }
  c->blob_bytes = B.size;
  for (u32 lvl = 1; lvl <= L; ++lvl) {
    LevelPlan& P = c->lv[lvl];
    uint8_t* d = c->blob;
    PlanDev pd{};
    pd.mu_jobs = (const ConvJobDev*)(d + P.o_mu_jobs); pd.mu_c = (const u32*)(d + P.o_mu_c);
    pd.md_jobs = (const ConvJobDev*)(d + P.o_md_jobs); pd.md_c = (const u32*)(d + P.o_md_c);
    pd.dt_mod = (const u32*)(d + P.o_dt_mod); pd.emod = (const u32*)(d + P.o_emod);
    pd.dtg_limb = (const u32*)(d + P.o_dtg_limb); pd.dtg_first = (const u32*)(d + P.o_dtg_first);
    pd.dtg_count = P.dtg_count;
    pd.y_mod = (const u32*)(d + P.o_y_mod); pd.y_scale = (const u64*)(d + P.o_y_scale);
    pd.s_mod = (const u32*)(d + P.o_s_mod); pd.s_scale = (const u64*)(d + P.o_s_scale);
    pd.qlinv = (const u64*)(d + P.o_qlinv); pd.qlmod = (const u64*)(d + P.o_qlmod);
    pd.pinv_l = P.pinv_l; pd.pinv_ls = shoup(P.pinv_l, q[lvl - 1]);
    pd.level = lvl; pd.beta = P.beta; pd.dt_limbs = P.dt_limbs;
    for (u32 j = 0; j < (u32)MAX_DIGITS; ++j) { pd.dt_first[j] = P.dt_first[j]; pd.lo[j] = P.lo[j]; pd.cnt[j] = P.cnt[j]; }
    memcpy(B.bytes.data() + P.o_plan, &pd, sizeof pd);
  }
  {
    hipError_t e = hipMemcpy(c->blob, B.bytes.data(), B.bytes.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(HE_EDEVICE, "table upload failed: %s", hipGetErrorString(e));
  }
  uint8_t* b = c->blob;
  c->mods = (const ModInfo*)(b + o_mods);
  c->tw = (const Tw2*)(b + o_tw);
  c->itw = (const Tw2*)(b + o_itw);
  c->gtw = (const double*)(b + o_gt);
  c->igtw = (const double*)(b + o_igt);
  c->gstride = (u32)gst;
  c->iota = (const u32*)(b + o_iota);
  c->spec_scale = (const u64*)(b + o_spec); c->pinv = (const u64*)(b + o_pinv);
  c->pmod = (const u64*)(b + o_pmod);
  for (u32 lvl = 1; lvl <= L; ++lvl) {
    LevelPlan& P = c->lv[lvl];
    P.modup_scale = (const u64*)(b + P.o_modup_scale);
    P.dt_mod = (const u32*)(b + P.o_dt_mod);
    P.emod = (const u32*)(b + P.o_emod);
    P.qlinv = (const u64*)(b + P.o_qlinv);
    P.qlmod = (const u64*)(b + P.o_qlmod);
    P.mu_c = (const u32*)(b + P.o_mu_c); P.md_c = (const u32*)(b + P.o_md_c);
    P.y_mod = (const u32*)(b + P.o_y_mod); P.y_scale = (const u64*)(b + P.o_y_scale);
    P.s_mod = (const u32*)(b + P.o_s_mod); P.s_scale = (const u64*)(b + P.o_s_scale);
    P.mu_jobs = (const ConvJobDev*)(b + P.o_mu_jobs); P.md_jobs = (const ConvJobDev*)(b + P.o_md_jobs);
    P.plan = (const PlanDev*)(b + P.o_plan);
  }
  *out = c.release();
  return HE_OK;
}

extern "C" {

size_t he_ctx_device_bytes(uint32_t log_n, uint32_t L, uint32_t K, uint32_t dnum, const uint64_t* q,
                           const uint64_t* p) {
  size_t n = 0;
  if (ctx_make(log_n, L, K, dnum, q, p, 0, true, nullptr, 0, &n, nullptr) != HE_OK) return 0;
  return n;
}

he_status he_ctx_create(uint32_t log_n, uint32_t L, uint32_t K, uint32_t dnum, const uint64_t* q,
                        const uint64_t* p, int device, void* d_tables, size_t tables_bytes, he_ctx** out) {
  if (!out) return fail(HE_EINVAL, "he_ctx_create: null pointer");
  return ctx_make(log_n, L, K, dnum, q, p, device, false, d_tables, tables_bytes, nullptr, out);
}

he_status he_ctx_create_w32(uint32_t log_n, uint32_t L, uint32_t K, uint32_t dnum, const uint64_t* q,
                            const uint64_t* p, int device, void* d_tables, size_t tables_bytes, he_ctx** out) {
  if (!out) return fail(HE_EINVAL, "he_ctx_create_w32: null pointer");
  return ctx_make(log_n, L, K, dnum, q, p, device, false, d_tables, tables_bytes, nullptr, out, true);
}

size_t he_ctx_table_bytes(const he_ctx* c) { return c ? c->blob_bytes : 0; }
uint32_t he_ctx_word_bytes(const he_ctx* c) { return c ? (c->w32 ? 4u : 8u) : 0u; }

void he_ctx_destroy(he_ctx* c) {
  if (!c) return;
  for (auto& r : c->trecs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->tpool) (void)hipEventDestroy(e);
  if (c->blob && c->owns_blob) {
    (void)hipSetDevice(c->device);
    (void)hipFree(c->blob);
  }
  delete c;
}

he_status he_ctx_info(const he_ctx* c, uint32_t* log_n, uint32_t* L, uint32_t* K, uint32_t* dnum,
                      uint64_t* moduli) {
  if (!c) return fail(HE_EINVAL, "null context");
  if (log_n) *log_n = c->log_n;
  if (L) *L = c->L;
  if (K) *K = c->K;
  if (dnum) *dnum = c->dnum;
  if (moduli) memcpy(moduli, c->mod.data(), c->mod.size() * sizeof(u64));
  return HE_OK;
}

size_t he_ct_bytes(const he_ctx* c, uint32_t level) { return c ? 2ull * level * c->N * word_bytes(c) : 0; }
size_t he_evk_bytes(const he_ctx* c) {
  return c ? (size_t)c->dnum * 2 * (c->L + c->K) * c->N * word_bytes(c) : 0;
}
size_t he_pk_bytes(const he_ctx* c) { return c ? 2ull * c->L * c->N * word_bytes(c) : 0; }

static size_t mul_ws_limbs(const he_ctx* c, u32 level) {
  const LevelPlan& P = c->lv[level];
  // D2, Y (+2), DT, KS (+1 per poly), Zp, Zc, RL
  return (size_t)level + (level + 2) + P.dt_limbs + 2 * (level + c->K + 1) + 2 * level + 2 * level + 2 * level;
}
static size_t keygen_ws_limbs(const he_ctx* c) {
  // S, S2, E (over L+K) + staging for small vectors (dnum+2 int64 vectors)
  return 3 * (size_t)(c->L + c->K) + c->dnum + 2;
}

size_t he_workspace_bytes(const he_ctx* c, uint32_t level) {
  if (!c || level < 1 || level > c->L) return 0;
  if (c->w32) return mul_ws_limbs(c, level) * c->N * 4;  // he_mul32 only
  size_t l = mul_ws_limbs(c, level);
  if (level == c->L) l = std::max(l, keygen_ws_limbs(c));
  l = std::max(l, 3 * (size_t)level + 4);  // encrypt / decrypt
  return l * c->N * 8;
}

he_status he_valu_peaks(int device, uint32_t blocks, uint32_t iters, double* rates, he_stream stream) {
  if (!rates || blocks == 0 || blocks > (1u << 16) || iters == 0 || iters > (1u << 20))
    return fail(HE_EINVAL, "he_valu_peaks: bad arguments");
  HIP_TRY(hipSetDevice(device));
  hipStream_t st = (hipStream_t)stream;
  uint64_t* sink = nullptr;
  HIP_TRY(hipMalloc(&sink, (size_t)blocks * ub::THREADS * sizeof(uint64_t)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  he_status r = HE_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) r = fail(HE_EDEVICE, "event creation");
  using KFn = void (*)(uint32_t, uint32_t, uint64_t*);
  const KFn fns[ub::KINDS] = {ub::k_peak_mad, ub::k_peak_mulhi, ub::k_peak_mullo, ub::k_peak_fma64, ub::k_peak_add};
  const double lane_ops = (double)blocks * ub::THREADS * iters * ub::CHAINS;
  for (int k = 0; k < ub::KINDS && r == HE_OK; ++k) {
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {  // the first launch also loads the kernel
      hipLaunchKernelGGL(fns[k], dim3(blocks), dim3(ub::THREADS), 0, st, iters, 0x9e3779b1u, sink);
      (void)hipEventRecord(e0, st);
      hipLaunchKernelGGL(fns[k], dim3(blocks), dim3(ub::THREADS), 0, st, iters, 0x9e3779b1u, sink);
      (void)hipEventRecord(e1, st);
      float ms = 0;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        r = fail(HE_EDEVICE, "he_valu_peaks: timing failed");
        break;
      }
      best = std::min(best, ms);
    }
    rates[k] = lane_ops / (best * 1e-3);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  if (r == HE_OK && hipGetLastError() != hipSuccess) r = fail(HE_EDEVICE, "he_valu_peaks: launch failed");
  return r;
}

size_t he_mul_noalloc_bytes(const he_ctx* c, uint32_t level) {
  if (!c || level < 1 || level > c->L) return 0;
  return mul_ws_limbs(c, level) * c->N * 8;
}

he_status he_mul_noalloc(he_ctx* c, uint32_t level, const uint64_t* ct1, const uint64_t* ct2, const uint64_t* evk,
                         uint64_t* relin, uint64_t* out, he_stream stream) {
  if (!c) return fail(HE_EINVAL, "he_mul_noalloc: null context");
  if (level < 1 || level > c->L) return fail(HE_ELEVEL, "he_mul_noalloc: level %u not in [1, L]", level);
  const size_t need = he_mul_noalloc_bytes(c, level);
  if (need > (size_t)HE_NOALLOC_SCRATCH_BYTES)
    return fail(HE_ENOMEM, "he_mul_noalloc: level %u at N = 2^%u needs %zu bytes of scratch, the maximum is %zu", level,
                c->log_n, need, (size_t)HE_NOALLOC_SCRATCH_BYTES);
  void* ws = g_scratch[c->device];  // set when the context was created on this device
  if (!ws) return fail(HE_EDEVICE, "he_mul_noalloc: no scratch address for device %d", c->device);
  return he_mul(c, level, ct1, ct2, evk, relin, out, ws, HE_NOALLOC_SCRATCH_BYTES, stream);
}

he_status he_ntt(he_ctx* c, uint64_t* d, uint32_t nlimbs, uint32_t first_mod, int inverse,
                 he_stream stream) {
  if (he_status r_ = need_w64(c, "he_ntt")) return r_;
  if (!c || !d) return fail(HE_EINVAL, "he_ntt: null pointer");
  if (first_mod + nlimbs > c->L + c->K) return fail(HE_EINVAL, "he_ntt: modulus range");
  HIP_TRY(hipSetDevice(c->device));
  ntt_launch(c, !inverse, d, d, c->N, c->N, 0, 0, c->iota + first_mod, nullptr, nlimbs, 1,
             (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- stage launches
namespace {

// Tile choices a batch may select: the defaults at every ring degree, and
// at N = 2^16 also 2048-element cols tiles and 1024-element blocks tiles.
bool tiles_supported(u32 log_n, TileCfg t) {
  if (t.fused_ip > (u32)IP_WAVES) return false;  // a digit threshold: pairs of >= fused_ip digits fuse
  if (t.logr != 0 && !(log_n == 16 && t.logr == 4)) return false;  // radix 16 at N = 2^16 only
  if (t.epw_c == EPW_C && t.epw_b == EPW_B) return true;
  return log_n == 16 && (t.epw_c == 2048 || t.epw_c == 4096) && (t.epw_b == 1024 || t.epw_b == 2048);
}

// Tiles of he_mul, he_rescale and new batches: at N = 2^16, 2048-element
// cols tiles and 1024-element blocks tiles (measured 3% and 1.5% faster
// per HE Mul: more workgroups for the one-round-deep passes), elsewhere
// the defaults.  The fused mod-up/inner-product pass is slower for a
// single HE Mul (measured 6%) and is left to the batch tuner.
TileCfg default_tiles(u32 log_n) {
  TileCfg t;
  if (log_n == 16) {
    t.epw_c = 2048;
    t.epw_b = 1024;
  }
  return t;
}

const char* stage_name(int s) {
  static const char* names[ST_COUNT + 3] = {"tensor_intt", "y_intt_cols", "modup_convert", "modup_ntt_cols",
                                            "modup_ntt_blocks", "inner_product", "special_intt_blocks",
                                            "modup_blocks_inner_product", "special_intt_cols", "moddown_convert",
                                            "moddown_lift_ntt_cols", "ntt_combine_rescale", "lift_ntt_cols",
                                            "ntt_rescale", "y_intt_blocks"};
  return names[s];
}

// Algorithmic work of one pair in a stage: (ops, bytes).  ops are
// butterflies for NTT passes (+N per limb for the inverse cols scaling),
// 64x64 multiply-accumulates for conversion and inner product, modular
// products for the element-wise parts; bytes are limbs read + written x 8N.
void stage_work(const he_ctx* c, int st, u32 level, bool rs, double& ops, double& bytes, bool wrl = true) {
  const LevelPlan& P = c->lv[level];
  const double N = (double)c->N, hN = N / 2, K = c->K, l = level, ex = rs ? 1 : 0;
  const int n1 = (int)c->log_n / 2, n2 = (int)c->log_n - n1;
  const double ne = l + K;
  double macs = 0;
  for (u32 j = 0; j < P.beta; ++j) macs += (double)P.cnt[j] * (ne - P.cnt[j]);
  switch (st) {
    case ST_TENSOR: ops = (l + 2 * ex) * hN * n2 + 4 * l * N; bytes = (4 * l + 3 * l + l + 2 * ex) * N * 8; break;
    case ST_Y_ICOLS: ops = (l + 2 * ex) * (hN * n1 + N); bytes = 2 * (l + 2 * ex) * N * 8; break;
    case ST_MU_CONV: ops = macs * N; bytes = (l + P.dt_limbs) * N * 8; break;
    case ST_DT_NCOLS: ops = P.dt_limbs * hN * n1; bytes = 2.0 * P.dt_limbs * N * 8; break;
    case ST_DT_NBLOCKS: ops = P.dt_limbs * hN * n2; bytes = 2.0 * P.dt_limbs * N * 8; break;
    case ST_IP:  // + the inverse blocks pass of the special limbs (and of limb level-1 when rescaling)
      ops = 2.0 * P.beta * ne * N + 2 * (K + ex) * hN * n2;
      bytes = (3.0 * P.beta + 2) * ne * N * 8 + 2 * ex * N * 8;
      break;
    case ST_KS_IBLOCKS: ops = bytes = 0; break;
    case ST_BLOCKS_IP:  // mod-up limbs (cols-pass form) and d2 in, evk in, ks out
      ops = P.dt_limbs * hN * n2 + 2.0 * P.beta * ne * N + 2 * (K + ex) * hN * n2;
      bytes = (P.dt_limbs + l + 2.0 * P.beta * ne + 2 * (ne + ex)) * N * 8;
      break;
    case ST_KS_ICOLS: ops = 2 * (K + ex) * (hN * n1 + N); bytes = 4 * (K + ex) * N * 8; break;
    case ST_MD_CONV: {  // special limbs in, z' out; rescaling: y, ks[level+K] in, r out or merged
      const double lo = (rs && !wrl) ? l - 1 : l;
      ops = 2 * K * l * N;
      bytes = (2 * K + 2 * lo + (rs ? (wrl ? 6 : 4) : 0)) * N * 8;
      break;
    }
    case ST_Z_NCOLS: {  // z' cols (z' + s when merged), plus the lift's cols pass when not merged
      const double lo = (rs && !wrl) ? l - 1 : l, ls = (rs && wrl) ? l - 1 : 0;
      ops = 2 * (lo + ls) * hN * n1;
      bytes = (4 * lo + (ls ? 2 * ls + 2 : 0)) * N * 8;
      break;
    }
    case ST_COMBINE: {  // z, ks, d in; out out when rescaling (s in when not merged); rl out when requested
      const double lo = (rs && !wrl) ? l - 1 : l;  // limbs combined
      ops = 2 * lo * hN * n2 + 2 * lo * N + (rs ? 2 * (l - 1) * ((wrl ? hN * n2 : 0) + N) : 0);
      bytes = (2 * lo * 3 + (wrl ? 2 * l : 0) + (rs ? 2 * (l - 1) * (wrl ? 2 : 1) : 0)) * N * 8;
      break;
    }
    case ST_LIFT: ops = rs ? 2 * (l - 1) * hN * n1 : 0; bytes = rs ? (2 * (l - 1) + 6) * N * 8 : 0; break;
    case ST_RESCALE: ops = rs ? 2 * (l - 1) * hN * n2 : 0; bytes = rs ? 2 * (l - 1) * 3 * N * 8 : 0; break;
    case ST_Y_IBLOCKS: ops = l * hN * n2; bytes = 2 * l * N * 8; break;
    default: ops = bytes = 0;
  }
}

void launch_stage(const he_ctx* c, int stage, const Common& cm, const Batch& b, double ops, double bytes,
                  hipStream_t st, TileCfg t = TileCfg{}) {
  if (!b.nitems) return;
  timed(c, stage_name(stage), ops, bytes, st, [&] {
    if (c->w32) {
      if (c->log_n <= 15) launch_w32_small(c->log_n, stage, cm, b, st);
      else launch_w32_n16(stage, cm, b, st);  // 32-bit-word contexts stop at N = 2^16
    }
    else if (c->log_n <= 15) launch_u64_small(c->log_n, stage, cm, b, st);
    else if (c->log_n == 16) launch_u64_n16(stage, cm, b, st, t);
    else launch_u64_n17(stage, cm, b, st);
  });
}

Common make_common(const he_ctx* c, const u64* evk) {
  Common cm{};
  cm.mods = c->mods; cm.tw = c->tw; cm.itw = c->itw; cm.evk = evk; cm.pinv = c->pinv; cm.iota = c->iota;
  cm.gtw = c->gtw; cm.igtw = c->igtw; cm.gstride = c->gstride;
  cm.L = c->L; cm.K = c->K; cm.log_n = c->log_n; cm.dnum = c->dnum;
  cm.bigq = 1;
  for (u64 m : c->mod) cm.bigq &= m >> 32 ? 1u : 0u;
  return cm;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  return (const uint8_t*)a < (const uint8_t*)b + nb && (const uint8_t*)b < (const uint8_t*)a + na;
}

// Lay out one pair's workspace starting at ws; returns limbs used (a limb
// is N words of the context's word size).
u64 pair_layout(const he_ctx* c, u32 level, void* ws, PairDesc& pd) {
  const LevelPlan& P = c->lv[level];
  const u64 lb = c->N * word_bytes(c);
  uint8_t* w = (uint8_t*)ws;
  u64 limbs = 0;
  auto take = [&](u64*& ptr, u64 n) {
    ptr = (u64*)(w + limbs * lb);
    limbs += n;
  };
  take(pd.d2, level);
  take(pd.y, level + 2);
  take(pd.dt, P.dt_limbs);
  take(pd.ks, 2ull * (level + c->K + 1));
  take(pd.z, 2ull * level);
  take(pd.zc, 2ull * level);
  return limbs;
}

}  // namespace

extern "C" {

}  // extern "C"

// HE Mul on stored words of either size (the context's): pointers are
// untyped bases of [2][level][N] words.
static he_status mul_impl(he_ctx* c, uint32_t level, const uint64_t* ct1, const uint64_t* ct2, const uint64_t* evk,
                          uint64_t* relin, uint64_t* out, void* ws, size_t ws_bytes, he_stream stream) {
  if (!c || !ct1 || !ct2 || !evk || !ws) return fail(HE_EINVAL, "he_mul: null pointer");
  if (!relin && !out) return fail(HE_EINVAL, "he_mul: no output requested");
  if (level < 1 || level > c->L) return fail(HE_ELEVEL, "he_mul: level %u not in [1, L]", level);
  if (out && level < 2) return fail(HE_ELEVEL, "he_mul: rescale needs level >= 2");
  const u64 wb = word_bytes(c);
  if (ws_bytes < mul_ws_limbs(c, level) * c->N * wb) return fail(HE_ENOMEM, "he_mul: workspace too small");
  const u64 N = c->N, ct_words = 2ull * level * N;
  for (const u64* o : {(const u64*)relin, (const u64*)out}) {
    if (!o) continue;
    if (overlaps(o, ct_words * wb, ct1, ct_words * wb) || overlaps(o, ct_words * wb, ct2, ct_words * wb))
      return fail(HE_EINVAL, "he_mul: output aliases an input");
  }
  if (relin && out && overlaps(relin, ct_words * wb, out, (ct_words - 2 * N) * wb))
    return fail(HE_EINVAL, "he_mul: the two outputs overlap");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const LevelPlan& P = c->lv[level];
  PairDesc pd{};
  pd.ct1 = ct1; pd.ct2 = ct2; pd.out = out; pd.r = nullptr; pd.plan = P.plan; pd.level = level;
  pd.rs = out ? 1 : 0;
  pd.wrl = relin ? 1 : 0;
  const u64 used = pair_layout(c, level, ws, pd);
  pd.rl = relin ? relin : (u64*)((uint8_t*)ws + used * c->N * word_bytes(c));
  const Common cm = make_common(c, evk);
  auto run = [&](int s, hipStream_t on) {
    Batch b{};
    b.one = pd;
    b.npairs = 1;
    b.nitems = stage_items(s, c->log_n, level, c->K, c->alpha, P.beta, P.dt_limbs, pd.rs != 0, pd.wrl != 0, default_tiles(c->log_n));
    double ops = 0, bytes = 0;
    if (c->timing) stage_work(c, s, level, pd.rs != 0, ops, bytes, pd.wrl != 0);
    launch_stage(c, s, cm, b, ops, bytes, on, default_tiles(c->log_n));
  };
  for (int s = 0; s < ST_COUNT; ++s) run(s, st);
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

extern "C" {

he_status he_mul(he_ctx* c, uint32_t level, const uint64_t* ct1, const uint64_t* ct2, const uint64_t* evk,
                 uint64_t* relin, uint64_t* out, void* ws, size_t ws_bytes, he_stream stream) {
  if (he_status r = need_w64(c, "he_mul")) return r;
  return mul_impl(c, level, ct1, ct2, evk, relin, out, ws, ws_bytes, stream);
}

he_status he_mul32(he_ctx* c, uint32_t level, const uint32_t* ct1, const uint32_t* ct2, const uint32_t* evk,
                   uint32_t* relin, uint32_t* out, void* ws, size_t ws_bytes, he_stream stream) {
  if (c && !c->w32) return fail(HE_EUNSUPPORTED, "he_mul32: the context stores 64-bit words (use he_mul)");
  return mul_impl(c, level, (const uint64_t*)ct1, (const uint64_t*)ct2, (const uint64_t*)evk, (uint64_t*)relin,
                  (uint64_t*)out, ws, ws_bytes, stream);
}

he_status he_rescale(he_ctx* c, uint32_t level, const uint64_t* d_in, uint64_t* d_out, void* ws,
                     size_t ws_bytes, he_stream stream) {
  if (he_status r_ = need_w64(c, "he_rescale")) return r_;
  if (!c || !d_in || !d_out || !ws) return fail(HE_EINVAL, "he_rescale: null pointer");
  if (level < 2 || level > c->L) return fail(HE_ELEVEL, "he_rescale: level %u not in [2, L]", level);
  if (ws_bytes < (2 + 2 * (size_t)level) * c->N * 8) return fail(HE_ENOMEM, "he_rescale: workspace too small");
  // one launch reads every input limb while others write output limbs
  if (overlaps(d_out, 2ull * (level - 1) * c->N * 8, d_in, 2ull * level * c->N * 8))
    return fail(HE_EINVAL, "he_rescale: output overlaps the input");
  if (overlaps(ws, ws_bytes, d_in, 2ull * level * c->N * 8) || overlaps(ws, ws_bytes, d_out, 2ull * (level - 1) * c->N * 8))
    return fail(HE_EINVAL, "he_rescale: workspace overlaps a ciphertext");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const u64 N = c->N;
  u64* R = (u64*)ws;
  // coefficient form of the dropped limb of both polynomials
  ntt_launch(c, false, d_in + (u64)(level - 1) * N, R, N, N, (u64)level * N, N, c->iota + (level - 1), nullptr, 1,
             2, st);
  const LevelPlan& P = c->lv[level];
  PairDesc pd{};
  pd.rl = const_cast<u64*>(d_in);  // read only by the rescale stages
  pd.out = d_out; pd.r = R; pd.d2 = R + 2 * N; pd.plan = P.plan; pd.level = level; pd.rs = 1;
  const Common cm = make_common(c, nullptr);
  for (int s : {(int)ST_LIFT, (int)ST_RESCALE}) {
    Batch b{};
    b.one = pd;
    b.npairs = 1;
    b.nitems = stage_items(s, c->log_n, level, c->K, c->alpha, P.beta, P.dt_limbs, true, false, default_tiles(c->log_n));
    double ops = 0, bytes = 0;
    if (c->timing) stage_work(c, s, level, true, ops, bytes);
    launch_stage(c, s, cm, b, ops, bytes, st, default_tiles(c->log_n));
  }
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

// ---- ciphertext descriptors: data plus level and scale (Sec. III-A)

he_status he_ct_import(he_ctx* c, const uint64_t* host, uint32_t level, double scale, he_ct* ct,
                       he_stream stream) {
  if (he_status r_ = need_w64(c, "he_ct_import")) return r_;
  if (!c || !host || !ct || !ct->data) return fail(HE_EINVAL, "he_ct_import: null pointer");
  if (level < 1 || level > c->L) return fail(HE_ELEVEL, "he_ct_import: level %u not in [1, L]", level);
  if (!(scale > 0) || !std::isfinite(scale)) return fail(HE_EINVAL, "he_ct_import: scale must be positive");
  const u64 N = c->N;
  for (u32 u = 0; u < 2; ++u)
    for (u32 i = 0; i < level; ++i) {
      const uint64_t* row = host + ((u64)u * level + i) * N;
      const u64 m = c->mod[i];
      for (u64 k = 0; k < N; ++k)
        if (row[k] >= m)
          return fail(HE_EINVAL, "he_ct_import: poly %u limb %u coefficient %llu is not below q_%u", u, i,
                      (unsigned long long)k, i);
    }
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpyAsync(ct->data, host, 2ull * level * N * 8, hipMemcpyHostToDevice, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  ct->level = level;
  ct->scale = scale;
  return HE_OK;
}

he_status he_ct_export(he_ctx* c, const he_ct* ct, uint64_t* host, he_stream stream) {
  if (he_status r_ = need_w64(c, "he_ct_export")) return r_;
  if (!c || !ct || !ct->data || !host) return fail(HE_EINVAL, "he_ct_export: null pointer");
  if (ct->level < 1 || ct->level > c->L) return fail(HE_ELEVEL, "he_ct_export: level %u not in [1, L]", ct->level);
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpyAsync(host, ct->data, 2ull * ct->level * c->N * 8, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return HE_OK;
}

he_status he_mul_ct(he_ctx* c, const uint64_t* d_evk, const he_ct* a, const he_ct* b, he_ct* relin, he_ct* out,
                    void* ws, size_t ws_bytes, he_stream stream) {
  if (!c || !a || !b) return fail(HE_EINVAL, "he_mul_ct: null pointer");
  if (a->level != b->level) return fail(HE_ELEVEL, "he_mul_ct: operand levels %u and %u differ", a->level, b->level);
  if ((relin && !relin->data) || (out && !out->data)) return fail(HE_EINVAL, "he_mul_ct: output without data");
  const uint32_t level = a->level;
  const he_status r = he_mul(c, level, a->data, b->data, d_evk, relin ? relin->data : nullptr,
                             out ? out->data : nullptr, ws, ws_bytes, stream);
  if (r != HE_OK) return r;
  const double sc = a->scale * b->scale;
  if (relin) { relin->level = level; relin->scale = sc; }
  if (out) { out->level = level - 1; out->scale = sc / (double)c->mod[level - 1]; }
  return HE_OK;
}

he_status he_rescale_ct(he_ctx* c, const he_ct* in, he_ct* out, void* ws, size_t ws_bytes, he_stream stream) {
  if (!c || !in || !out || !out->data) return fail(HE_EINVAL, "he_rescale_ct: null pointer");
  const he_status r = he_rescale(c, in->level, in->data, out->data, ws, ws_bytes, stream);
  if (r != HE_OK) return r;
  out->level = in->level - 1;
  out->scale = in->scale / (double)c->mod[in->level - 1];
  return HE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batches
// A batch owns device descriptors (one PairDesc per pair, then per stage the
// prefix sums of the pairs' work items for the current tiles) and a
// schedule: NTT tiles and a split of the pairs into `chunks` contiguous
// groups whose stage chains alternate between the caller's stream and a side
// stream (fork/join by events, also inside a captured graph), so that stages
// of different groups overlap on the device.
struct he_batch {
  he_ctx* ctx = nullptr;
  u32 n = 0;
  void* dev = nullptr;                 // descriptors + offsets (device)
  bool owns_dev = true;                // false: caller-provided descriptor memory
  std::vector<uint8_t> host;           // staging copy (kept until destroy for async uploads)
  const PairDesc* pairs = nullptr;
  const u32* offs[ST_COUNT] = {};
  std::vector<u32> hoffs;              // host copy of the offsets [ST_COUNT][n + 1]
  u32 nitems[ST_COUNT] = {};
  std::vector<u32> levels;
  std::vector<uint8_t> rs, wrl;
  TileCfg tiles{};
  u32 chunks = 1;
  std::vector<u32> cut{};              // chunk boundaries in pairs [chunks + 1]
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  u32 stamp = 0;                       // bumped when the schedule changes
  u32 group_stamp = 0;                 // stamp a batch group's graph was captured with
  // cached graph of the whole batched HE Mul
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const u64* graph_evk = nullptr;
};

static size_t batch_ws_words(const he_ctx* c, const he_batch_item* items, u32 n) {
  size_t w = 0;
  for (u32 i = 0; i < n; ++i) {
    PairDesc tmp{};
    w += pair_layout(c, items[i].level, nullptr, tmp) * c->N;
    if (!items[i].relin) w += 2ull * items[i].level * c->N;
  }
  return w;
}

// Per-stage item prefix sums of the batch for its current tiles, into
// bt->hoffs, bt->nitems and the offsets part of the staging buffer.
static he_status batch_offsets(const he_ctx* c, he_batch* bt) {
  const u32 n = bt->n;
  bt->hoffs.assign((size_t)ST_COUNT * (n + 1), 0);
  for (int s = 0; s < ST_COUNT; ++s) {
    u64 acc = 0;
    for (u32 i = 0; i < n; ++i) {
      bt->hoffs[(size_t)s * (n + 1) + i] = (u32)acc;
      const LevelPlan& P = c->lv[bt->levels[i]];
      acc += stage_items(s, c->log_n, bt->levels[i], c->K, c->alpha, P.beta, P.dt_limbs, bt->rs[i] != 0, bt->wrl[i] != 0, bt->tiles);
    }
    if (acc > 0xffffff00ull) return fail(HE_EUNSUPPORTED, "he_batch: batch too large");
    bt->hoffs[(size_t)s * (n + 1) + n] = (u32)acc;
    bt->nitems[s] = (u32)acc;
  }
  memcpy(bt->host.data() + sizeof(PairDesc) * n, bt->hoffs.data(), sizeof(u32) * bt->hoffs.size());
  return HE_OK;
}

// Chunk boundaries with about equal sums of levels per chunk.
static void batch_cuts(he_batch* bt) {
  u64 tot = 0;
  for (u32 l : bt->levels) tot += l;
  bt->cut.assign(1, 0);
  u64 acc = 0;
  for (u32 i = 0; i < bt->n && bt->cut.size() < bt->chunks; ++i) {
    acc += bt->levels[i];
    if (acc * bt->chunks >= tot * bt->cut.size() && i + 1 < bt->n) bt->cut.push_back(i + 1);
  }
  bt->cut.push_back(bt->n);
}

extern "C" {

size_t he_batch_workspace_bytes(const he_ctx* c, const he_batch_item* items, uint32_t n) {
  if (!c || (!items && n)) return 0;
  return batch_ws_words(c, items, n) * 8;
}

size_t he_batch_desc_bytes(uint32_t n) {
  return (sizeof(PairDesc) * (size_t)n + sizeof(u32) * (size_t)ST_COUNT * (n + 1) + 255) & ~size_t(255);
}

static he_status batch_build(he_ctx* c, const he_batch_item* items, uint32_t n, void* ws, size_t ws_bytes,
                             std::unique_ptr<he_batch>& bt) {
  if (!c || !items || !ws || n == 0) return fail(HE_EINVAL, "he_batch_create: bad arguments");
  if (he_status r_ = need_w64(c, "he_batch_create")) return r_;
  for (u32 i = 0; i < n; ++i) {
    const he_batch_item& it = items[i];
    if (!it.ct1 || !it.ct2 || (!it.relin && !it.out)) return fail(HE_EINVAL, "he_batch_create: item %u incomplete", i);
    if (it.level < 1 || it.level > c->L) return fail(HE_ELEVEL, "he_batch_create: item %u level %u", i, it.level);
    if (it.out && it.level < 2) return fail(HE_ELEVEL, "he_batch_create: item %u: rescale needs level >= 2", i);
  }
  if (ws_bytes < batch_ws_words(c, items, n) * 8) return fail(HE_ENOMEM, "he_batch_create: workspace too small");
  bt.reset(new he_batch);
  bt->ctx = c;
  bt->n = n;
  bt->tiles = default_tiles(c->log_n);
  std::vector<PairDesc> pds(n);
  u64* w = (u64*)ws;
  for (u32 i = 0; i < n; ++i) {
    const he_batch_item& it = items[i];
    PairDesc& pd = pds[i];
    pd.ct1 = it.ct1; pd.ct2 = it.ct2; pd.out = it.out; pd.r = nullptr;
    pd.plan = c->lv[it.level].plan; pd.level = it.level; pd.rs = it.out ? 1 : 0; pd.wrl = it.relin ? 1 : 0;
    w += pair_layout(c, it.level, w, pd) * c->N;
    if (it.relin) {
      pd.rl = it.relin;
    } else {
      pd.rl = w;
      w += 2ull * it.level * c->N;
    }
    bt->levels.push_back(it.level);
    bt->rs.push_back(pd.rs);
    bt->wrl.push_back(pd.wrl);
  }
  const size_t pbytes = sizeof(PairDesc) * n, obytes = sizeof(u32) * (size_t)ST_COUNT * (n + 1);
  bt->host.resize(pbytes + obytes);
  memcpy(bt->host.data(), pds.data(), pbytes);
  batch_cuts(bt.get());
  return batch_offsets(c, bt.get());
}

static void batch_bind(he_batch* bt, void* dev) {
  bt->dev = dev;
  bt->pairs = (const PairDesc*)dev;
  const size_t pbytes = sizeof(PairDesc) * bt->n;
  for (int s = 0; s < ST_COUNT; ++s)
    bt->offs[s] = (const u32*)((uint8_t*)dev + pbytes) + (size_t)s * (bt->n + 1);
}

he_status he_batch_create(he_ctx* c, const he_batch_item* items, uint32_t n, void* ws, size_t ws_bytes,
                          he_batch** out) {
  if (!out) return fail(HE_EINVAL, "he_batch_create: null output");
  *out = nullptr;
  std::unique_ptr<he_batch> bt;
  he_status r = batch_build(c, items, n, ws, ws_bytes, bt);
  if (r != HE_OK) return r;
  HIP_TRY(hipSetDevice(c->device));
  void* dev = nullptr;
  HIP_TRY(hipMalloc(&dev, bt->host.size()));
  const hipError_t e = hipMemcpy(dev, bt->host.data(), bt->host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dev);
    return fail(HE_EDEVICE, "he_batch_create: upload failed: %s", hipGetErrorString(e));
  }
  batch_bind(bt.get(), dev);
  *out = bt.release();
  return HE_OK;
}

he_status he_batch_create_async(he_ctx* c, const he_batch_item* items, uint32_t n, void* ws, size_t ws_bytes,
                                void* d_desc, size_t desc_bytes, he_stream stream, he_batch** out) {
  if (!out || !d_desc) return fail(HE_EINVAL, "he_batch_create_async: null pointer");
  *out = nullptr;
  if (desc_bytes < he_batch_desc_bytes(n)) return fail(HE_ENOMEM, "he_batch_create_async: descriptor memory too small");
  std::unique_ptr<he_batch> bt;
  he_status r = batch_build(c, items, n, ws, ws_bytes, bt);
  if (r != HE_OK) return r;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpyAsync(d_desc, bt->host.data(), bt->host.size(), hipMemcpyHostToDevice, (hipStream_t)stream));
  bt->owns_dev = false;
  batch_bind(bt.get(), d_desc);
  *out = bt.release();
  return HE_OK;
}

static void batch_drop_graph(he_batch* bt) {
  if (bt->exec) { (void)hipGraphExecDestroy(bt->exec); bt->exec = nullptr; }
  if (bt->graph) { (void)hipGraphDestroy(bt->graph); bt->graph = nullptr; }
  bt->graph_evk = nullptr;
}

he_status he_batch_set_sched(he_batch* bt, const he_batch_sched* sc, he_stream stream) {
  if (!bt || !sc) return fail(HE_EINVAL, "he_batch_set_sched: null pointer");
  he_ctx* c = bt->ctx;
  TileCfg t;
  t.epw_c = sc->cols_tile;
  t.epw_b = sc->blocks_tile;
  t.fused_ip = sc->ip_fused;
  // radix 0 or the default radix of the passes: default; 16 at N = 2^16: log2 4
  const u32 dflt = 1u << radix_log((int)(c->log_n / 2));
  t.logr = (sc->radix == 0 || sc->radix == dflt) ? 0 : (sc->radix == 16 ? 4 : 99);
  if (!tiles_supported(c->log_n, t))
    return fail(HE_EUNSUPPORTED, "he_batch_set_sched: tiles %u/%u, radix %u not available at N = 2^%u", t.epw_c,
                t.epw_b, sc->radix, c->log_n);
  if (t.fused_ip && c->dnum > (u32)IP_WAVES)
    return fail(HE_EUNSUPPORTED, "he_batch_set_sched: the fused inner product takes at most %d digits", IP_WAVES);
  if (sc->chunks < 1 || sc->chunks > 8 || sc->chunks > bt->n)
    return fail(HE_EINVAL, "he_batch_set_sched: chunks %u not in [1, min(8, pairs)]", sc->chunks);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(st));  // the staging buffer may still feed an earlier upload
  bt->tiles = t;
  bt->chunks = sc->chunks;
  batch_cuts(bt);
  he_status r = batch_offsets(c, bt);
  if (r != HE_OK) return r;
  const size_t pbytes = sizeof(PairDesc) * bt->n;
  HIP_TRY(hipMemcpyAsync((uint8_t*)bt->dev + pbytes, bt->host.data() + pbytes, bt->host.size() - pbytes,
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (bt->chunks > 1 && !bt->side) {
    HIP_TRY(hipStreamCreateWithFlags(&bt->side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&bt->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&bt->ev_join, hipEventDisableTiming));
  }
  batch_drop_graph(bt);
  ++bt->stamp;  // graphs of batch groups holding this batch are recaptured
  return HE_OK;
}

he_status he_batch_get_sched(const he_batch* bt, he_batch_sched* sc) {
  if (!bt || !sc) return fail(HE_EINVAL, "he_batch_get_sched: null pointer");
  sc->cols_tile = bt->tiles.epw_c;
  sc->blocks_tile = bt->tiles.epw_b;
  sc->chunks = bt->chunks;
  sc->ip_fused = bt->tiles.fused_ip;
  sc->radix = bt->tiles.logr ? 1u << bt->tiles.logr : 1u << radix_log((int)(bt->ctx->log_n / 2));
  return HE_OK;
}

}  // extern "C"

// The 13 stages of pairs [p0, p1) on stream st.
static void batch_chain(he_ctx* c, he_batch* bt, const Common& cm, u32 p0, u32 p1, hipStream_t st) {
  const u32 n = bt->n;
  for (int s = 0; s < ST_COUNT; ++s) {
    Batch b{};
    b.pairs = bt->pairs + p0;
    b.offs = bt->offs[s] + p0;
    b.npairs = p1 - p0;
    b.nitems = bt->hoffs[(size_t)s * (n + 1) + p1] - bt->hoffs[(size_t)s * (n + 1) + p0];
    double ops = 0, bytes = 0;
    if (c->timing)
      for (u32 i = p0; i < p1; ++i) {
        double o = 0, by = 0;
        stage_work(c, s, bt->levels[i], bt->rs[i] != 0, o, by, bt->wrl[i] != 0);
        ops += o;
        bytes += by;
      }
    launch_stage(c, s, cm, b, ops, bytes, st, bt->tiles);
  }
}

static hipError_t batch_launch_all(he_ctx* c, he_batch* bt, const u64* evk, hipStream_t st) {
  const Common cm = make_common(c, evk);
  if (bt->chunks <= 1) {
    batch_chain(c, bt, cm, 0, bt->n, st);
    return hipGetLastError();
  }
  hipError_t e = hipEventRecord(bt->ev_fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(bt->side, bt->ev_fork, 0);
  if (e != hipSuccess) return e;
  for (u32 k = 0; k + 1 < bt->cut.size(); ++k)
    batch_chain(c, bt, cm, bt->cut[k], bt->cut[k + 1], (k & 1) ? bt->side : st);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(bt->ev_join, bt->side);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, bt->ev_join, 0);
  return e;
}

extern "C" {

he_status he_mul_batch(he_ctx* c, he_batch* bt, const uint64_t* evk, int use_graph, he_stream stream) {
  if (!c || !bt || !evk || bt->ctx != c) return fail(HE_EINVAL, "he_mul_batch: bad arguments");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  if (!use_graph || c->timing) {
    const hipError_t e = batch_launch_all(c, bt, evk, st);
    if (e != hipSuccess) return fail(HE_EDEVICE, "he_mul_batch: launch failed: %s", hipGetErrorString(e));
    return HE_OK;
  }
  if (!bt->exec || bt->graph_evk != evk) {
    batch_drop_graph(bt);
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t le = batch_launch_all(c, bt, evk, cap);
      e = hipStreamEndCapture(cap, &bt->graph);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
      batch_drop_graph(bt);
      return fail(HE_EDEVICE, "he_mul_batch: graph capture failed: %s", hipGetErrorString(e));
    }
    bt->graph_evk = evk;
  }
  HIP_TRY(hipGraphLaunch(bt->exec, st));
  return HE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batch groups
// Batches of different contexts (ring sizes) run as one unit: batch 0 on
// the caller's stream, batch i > 0 on a stream of the group, forked from
// and joined back to the caller's stream by events, so the rings' stage
// kernels overlap on the device; captured once into a single HIP graph.
struct he_batch_group {
  std::vector<he_batch*> batches;
  std::vector<hipStream_t> side;     // [n - 1]
  std::vector<hipEvent_t> ev_join;   // [n - 1]
  hipEvent_t ev_fork = nullptr;
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const u64*> graph_evks;
};

static void group_drop_graph(he_batch_group* g) {
  if (g->exec) { (void)hipGraphExecDestroy(g->exec); g->exec = nullptr; }
  if (g->graph) { (void)hipGraphDestroy(g->graph); g->graph = nullptr; }
  g->graph_evks.clear();
}

static hipError_t group_launch_all(he_batch_group* g, const uint64_t* const* evks, hipStream_t st) {
  const u32 n = (u32)g->batches.size();
  hipError_t e = hipSuccess;
  if (n > 1) {
    e = hipEventRecord(g->ev_fork, st);
    for (u32 i = 1; i < n && e == hipSuccess; ++i) e = hipStreamWaitEvent(g->side[i - 1], g->ev_fork, 0);
  }
  for (u32 i = 0; i < n && e == hipSuccess; ++i) {
    he_batch* bt = g->batches[i];
    e = batch_launch_all(bt->ctx, bt, evks[i], i ? g->side[i - 1] : st);
  }
  for (u32 i = 1; i < n && e == hipSuccess; ++i) {
    e = hipEventRecord(g->ev_join[i - 1], g->side[i - 1]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, g->ev_join[i - 1], 0);
  }
  return e;
}

extern "C" {

he_status he_batch_group_create(he_batch* const* batches, uint32_t n, he_batch_group** out) {
  if (!out || !batches || n == 0 || n > 64) return fail(HE_EINVAL, "he_batch_group_create: bad arguments");
  *out = nullptr;
  for (u32 i = 0; i < n; ++i) {
    if (!batches[i]) return fail(HE_EINVAL, "he_batch_group_create: batch %u is null", i);
    if (batches[i]->ctx->device != batches[0]->ctx->device)
      return fail(HE_EINVAL, "he_batch_group_create: batches on different devices");
    for (u32 j = 0; j < i; ++j)
      if (batches[j] == batches[i]) return fail(HE_EINVAL, "he_batch_group_create: batch %u listed twice", i);
  }
  for (u32 i = 0; i < n; ++i)
    if (batches[i]->chunks > 1)
      return fail(HE_EUNSUPPORTED, "he_batch_group_create: batch %u runs in %u chunks; a group takes one-chunk batches",
                  i, batches[i]->chunks);
  std::unique_ptr<he_batch_group, void (*)(he_batch_group*)> g(new he_batch_group, he_batch_group_destroy);
  g->batches.assign(batches, batches + n);
  for (he_batch* bt : g->batches) bt->group_stamp = bt->stamp;
  g->device = batches[0]->ctx->device;
  HIP_TRY(hipSetDevice(g->device));
  HIP_TRY(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
  for (u32 i = 1; i < n; ++i) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    g->side.push_back(s);
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    g->ev_join.push_back(e);
  }
  *out = g.release();
  return HE_OK;
}

he_status he_mul_batch_group(he_batch_group* g, const uint64_t* const* d_evks, int use_graph, he_stream stream) {
  if (!g || !d_evks) return fail(HE_EINVAL, "he_mul_batch_group: null pointer");
  const u32 n = (u32)g->batches.size();
  for (u32 i = 0; i < n; ++i) {
    if (!d_evks[i]) return fail(HE_EINVAL, "he_mul_batch_group: evk %u is null", i);
    if (g->batches[i]->group_stamp != g->batches[i]->stamp)
      return fail(HE_EUNSUPPORTED, "he_mul_batch_group: batch %u changed its schedule after the group was made", i);
  }
  HIP_TRY(hipSetDevice(g->device));
  hipStream_t st = (hipStream_t)stream;
  bool timing = false;
  for (he_batch* bt : g->batches) timing = timing || bt->ctx->timing;
  if (!use_graph || timing) {
    const hipError_t e = group_launch_all(g, d_evks, st);
    if (e != hipSuccess) return fail(HE_EDEVICE, "he_mul_batch_group: launch failed: %s", hipGetErrorString(e));
    return HE_OK;
  }
  const std::vector<const u64*> evks(d_evks, d_evks + n);
  if (!g->exec || g->graph_evks != evks) {
    group_drop_graph(g);
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t le = group_launch_all(g, d_evks, cap);
      e = hipStreamEndCapture(cap, &g->graph);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
      group_drop_graph(g);
      return fail(HE_EDEVICE, "he_mul_batch_group: graph capture failed: %s", hipGetErrorString(e));
    }
    g->graph_evks = evks;
  }
  HIP_TRY(hipGraphLaunch(g->exec, st));
  return HE_OK;
}

void he_batch_group_destroy(he_batch_group* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  for (hipStream_t s : g->side) (void)hipStreamSynchronize(s);
  group_drop_graph(g);
  for (hipStream_t s : g->side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : g->ev_join) (void)hipEventDestroy(e);
  if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
  delete g;
}

// Times `reps` graph replays of the batch under each candidate schedule and
// keeps the fastest: first the tiles (one chunk), then the chunk count with
// the best tiles.
he_status he_batch_autotune(he_ctx* c, he_batch* bt, const uint64_t* evk, uint32_t reps, he_stream stream,
                            he_batch_sched* best, double* best_ms) {
  if (!c || !bt || !evk || bt->ctx != c || reps == 0) return fail(HE_EINVAL, "he_batch_autotune: bad arguments");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto run = [&](const he_batch_sched& sc, double& ms) -> he_status {
    he_status r = he_batch_set_sched(bt, &sc, stream);
    if (r != HE_OK) return r;
    r = he_mul_batch(c, bt, evk, 1, stream);  // capture and warm up
    if (r != HE_OK) return r;
    HIP_TRY(hipEventRecord(e0, st));
    for (u32 i = 0; i < reps; ++i) {
      r = he_mul_batch(c, bt, evk, 1, stream);
      if (r != HE_OK) return r;
    }
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    ms = t / reps;
    return HE_OK;
  };
  std::vector<he_batch_sched> tiles;
  const TileCfg d = default_tiles(c->log_n);
  tiles.push_back({d.epw_c, d.epw_b, 1, 0, 0});
  if (c->log_n == 16)  // every tile pair at the default radix (8) and at radix 16
    for (uint32_t rdx : {0u, 16u})
      for (uint32_t ec : {4096u, 2048u})
        for (uint32_t eb : {2048u, 1024u})
          if (!(ec == d.epw_c && eb == d.epw_b && rdx == 0)) tiles.push_back({ec, eb, 1, 0, rdx});
  he_batch_sched b = tiles[0];
  double bms = 1e30;
  he_status r = HE_OK;
  for (const auto& sc : tiles) {
    double ms = 0;
    if ((r = run(sc, ms)) != HE_OK) break;
    if (ms < bms) { bms = ms; b = sc; }
  }
  // the fused mod-up blocks + inner product pass for the pairs of at least
  // 1, 2 or 3 digits (at its own radix; the other passes keep the chosen one)
  const he_batch_sched plain = b;
  for (uint32_t f = 1; f <= std::min(3u, c->dnum); ++f) {
    if (r != HE_OK || c->dnum > (u32)IP_WAVES) break;
    he_batch_sched sc = plain;
    sc.ip_fused = f;
    double ms = 0;
    if ((r = run(sc, ms)) == HE_OK && ms < bms) { bms = ms; b = sc; }
  }
  for (uint32_t ch : {2u, 4u}) {
    if (r != HE_OK || ch > bt->n) break;
    he_batch_sched sc = b;
    sc.chunks = ch;
    double ms = 0;
    if ((r = run(sc, ms)) != HE_OK) break;
    if (ms < bms) { bms = ms; b = sc; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r != HE_OK) return r;
  r = he_batch_set_sched(bt, &b, stream);
  if (r != HE_OK) return r;
  if (best) (void)he_batch_get_sched(bt, best);  // as get_sched reports it (default radix by value)
  if (best_ms) *best_ms = bms;
  return HE_OK;
}

void he_batch_destroy(he_batch* bt) {
  if (!bt) return;
  (void)hipSetDevice(bt->ctx->device);
  batch_drop_graph(bt);
  if (bt->side) (void)hipStreamSynchronize(bt->side);
  if (bt->ev_fork) (void)hipEventDestroy(bt->ev_fork);
  if (bt->ev_join) (void)hipEventDestroy(bt->ev_join);
  if (bt->side) (void)hipStreamDestroy(bt->side);
  if (bt->dev && bt->owns_dev) (void)hipFree(bt->dev);
  delete bt;
}

}  // extern "C"

extern "C" {

// ---------------------------------------------------------------- keys & encryption
static he_status upload_sync(void* dst, const void* src, size_t bytes, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return HE_OK;
}

he_status he_keygen(he_ctx* c, const int64_t* s, const int64_t* e_pk, const uint64_t* a_pk,
                    const int64_t* e_evk, const uint64_t* a_evk, uint64_t* d_pk, uint64_t* d_evk,
                    void* ws, size_t ws_bytes, he_stream stream) {
  if (he_status r_ = need_w64(c, "he_keygen")) return r_;
  if (!c || !s || !e_pk || !a_pk || !e_evk || !a_evk || !d_pk || !d_evk || !ws)
    return fail(HE_EINVAL, "he_keygen: null pointer");
  if (ws_bytes < keygen_ws_limbs(c) * c->N * 8) return fail(HE_ENOMEM, "he_keygen: workspace too small");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const u64 N = c->N;
  const u32 L = c->L, K = c->K, nm = L + K;
  u64* w = (u64*)ws;
  u64* S = w;  w += (u64)nm * N;
  u64* S2 = w; w += (u64)nm * N;
  u64* E = w;  w += (u64)nm * N;
  int64_t* sv = (int64_t*)w;             // [N]
  int64_t* ev = sv + N;                  // [N]
  int64_t* eev = ev + N;                 // [dnum][N]
  he_status r;
  if ((r = upload_sync(sv, s, N * 8, st)) != HE_OK) return r;
  if ((r = upload_sync(ev, e_pk, N * 8, st)) != HE_OK) return r;
  if ((r = upload_sync(eev, e_evk, (u64)c->dnum * N * 8, st)) != HE_OK) return r;
  // pk over q_0..q_{L-1}: a (host) -> d_pk poly 1
  if ((r = upload_sync(d_pk + (u64)L * N, a_pk, (u64)L * N * 8, st)) != HE_OK) return r;
  hipLaunchKernelGGL(k_small_to_limbs, ew_grid((u64)nm * N), dim3(EW_THREADS), 0, st, sv, S, c->iota, c->mods,
                     nm, c->log_n);
  ntt_launch(c, true, S, S, N, N, 0, 0, c->iota, nullptr, nm, 1, st);
  hipLaunchKernelGGL(k_small_to_limbs, ew_grid((u64)L * N), dim3(EW_THREADS), 0, st, ev, E, c->iota, c->mods,
                     L, c->log_n);
  ntt_launch(c, true, E, E, N, N, 0, 0, c->iota, nullptr, L, 1, st);
  hipLaunchKernelGGL(k_mul_add, ew_grid((u64)L * N), dim3(EW_THREADS), 0, st, d_pk + (u64)L * N, S, E, d_pk,
                     c->iota, c->mods, L, c->log_n);
  // evk
  hipLaunchKernelGGL(k_mul, ew_grid((u64)nm * N), dim3(EW_THREADS), 0, st, S, S, S2, c->iota, c->mods, nm,
                     c->log_n);
  for (u32 j = 0; j < c->dnum; ++j) {
    u64* bj = d_evk + (u64)j * 2 * nm * N;
    u64* aj = bj + (u64)nm * N;
    if ((r = upload_sync(aj, a_evk + (u64)j * nm * N, (u64)nm * N * 8, st)) != HE_OK) return r;
    hipLaunchKernelGGL(k_small_to_limbs, ew_grid((u64)nm * N), dim3(EW_THREADS), 0, st, eev + (u64)j * N, E,
                       c->iota, c->mods, nm, c->log_n);
    ntt_launch(c, true, E, E, N, N, 0, 0, c->iota, nullptr, nm, 1, st);
    const u32 dlo = j * c->alpha, dhi = std::min(L, (j + 1) * c->alpha);
    hipLaunchKernelGGL(k_evk_b, ew_grid((u64)nm * N), dim3(EW_THREADS), 0, st, aj, S, S2, E, bj, c->pmod,
                       c->mods, nm, dlo, dhi, c->log_n);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return HE_OK;
}

he_status he_encrypt(he_ctx* c, uint32_t level, const int64_t* m, const int64_t* v, const int64_t* e0,
                     const int64_t* e1, const uint64_t* d_pk, uint64_t* d_ct, void* ws, size_t ws_bytes,
                     he_stream stream) {
  if (he_status r_ = need_w64(c, "he_encrypt")) return r_;
  if (!c || !m || !v || !e0 || !e1 || !d_pk || !d_ct || !ws) return fail(HE_EINVAL, "he_encrypt: null pointer");
  if (level < 1 || level > c->L) return fail(HE_ELEVEL, "he_encrypt: level %u not in [1, L]", level);
  if (ws_bytes < (3 * (size_t)level + 4) * c->N * 8) return fail(HE_ENOMEM, "he_encrypt: workspace too small");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const u64 N = c->N, tot = (u64)level * N;
  u64* w = (u64*)ws;
  u64* V = w;  w += tot;
  u64* T0 = w; w += tot;
  u64* T1 = w; w += tot;
  int64_t* hv = (int64_t*)w;
  he_status r;
  if ((r = upload_sync(hv, v, N * 8, st)) != HE_OK) return r;
  if ((r = upload_sync(hv + N, e0, N * 8, st)) != HE_OK) return r;
  if ((r = upload_sync(hv + 2 * N, m, N * 8, st)) != HE_OK) return r;
  if ((r = upload_sync(hv + 3 * N, e1, N * 8, st)) != HE_OK) return r;
  auto to_ntt = [&](const int64_t* src, u64* dst) {
    hipLaunchKernelGGL(k_small_to_limbs, ew_grid(tot), dim3(EW_THREADS), 0, st, src, dst, c->iota, c->mods,
                       level, c->log_n);
    ntt_launch(c, true, dst, dst, N, N, 0, 0, c->iota, nullptr, level, 1, st);
  };
  to_ntt(hv, V);
  // T0 = NTT(e0 mod q + m mod q): expand both, add, transform
  hipLaunchKernelGGL(k_small_to_limbs, ew_grid(tot), dim3(EW_THREADS), 0, st, hv + N, T0, c->iota, c->mods,
                     level, c->log_n);
  hipLaunchKernelGGL(k_small_to_limbs, ew_grid(tot), dim3(EW_THREADS), 0, st, hv + 2 * N, T1, c->iota, c->mods,
                     level, c->log_n);
  hipLaunchKernelGGL(k_add, ew_grid(tot), dim3(EW_THREADS), 0, st, T0, T1, T0, c->iota, c->mods, level,
                     c->log_n);
  ntt_launch(c, true, T0, T0, N, N, 0, 0, c->iota, nullptr, level, 1, st);
  to_ntt(hv + 3 * N, T1);
  hipLaunchKernelGGL(k_mul_add, ew_grid(tot), dim3(EW_THREADS), 0, st, V, d_pk, T0, d_ct, c->iota, c->mods,
                     level, c->log_n);
  hipLaunchKernelGGL(k_mul_add, ew_grid(tot), dim3(EW_THREADS), 0, st, V, d_pk + (u64)c->L * N, T1,
                     d_ct + tot, c->iota, c->mods, level, c->log_n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return HE_OK;
}

he_status he_decrypt(he_ctx* c, uint32_t level, const uint64_t* d_ct, const int64_t* s, uint64_t* d_m,
                     void* ws, size_t ws_bytes, he_stream stream) {
  if (he_status r_ = need_w64(c, "he_decrypt")) return r_;
  if (!c || !d_ct || !s || !d_m || !ws) return fail(HE_EINVAL, "he_decrypt: null pointer");
  if (level < 1 || level > c->L) return fail(HE_ELEVEL, "he_decrypt: level %u not in [1, L]", level);
  if (ws_bytes < ((size_t)level + 1) * c->N * 8) return fail(HE_ENOMEM, "he_decrypt: workspace too small");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const u64 N = c->N, tot = (u64)level * N;
  u64* S = (u64*)ws;
  int64_t* sv = (int64_t*)(S + tot);
  he_status r;
  if ((r = upload_sync(sv, s, N * 8, st)) != HE_OK) return r;
  hipLaunchKernelGGL(k_small_to_limbs, ew_grid(tot), dim3(EW_THREADS), 0, st, sv, S, c->iota, c->mods, level,
                     c->log_n);
  ntt_launch(c, true, S, S, N, N, 0, 0, c->iota, nullptr, level, 1, st);
  hipLaunchKernelGGL(k_dec, ew_grid(tot), dim3(EW_THREADS), 0, st, d_ct, S, d_m, c->mods, level, c->log_n);
  ntt_launch(c, false, d_m, d_m, N, N, 0, 0, c->iota, nullptr, level, 1, st);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return HE_OK;
}

}  // extern "C"
#include "big_host.hpp"
#include "scheme_host.hpp"
