/*
 * he_oracle.c -- plain, slow, obviously-correct CPU oracle for full-RNS
 * CKKS (HEAAN) HE Mul.  TEST INFRASTRUCTURE ONLY: only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the HIP library.
 *
 * Every modular product is computed as ((unsigned __int128)a * b) % m: no
 * Shoup, Barrett or Montgomery reduction, no lazy ranges, no fusion.  Every
 * stored residue is canonical, in [0, m).
 *
 * Paper: "HEAAN Demystified" (arXiv 2003.04510).
 *   - NTT: the negacyclic transform of Sec. IV (values at the odd powers of
 *     the 2N-th root psi, bit-reversed order, the map Algorithms 3-4
 *     compute), written as the recursive Chinese-remainder split of
 *     X^N + 1; iNTT: each split undone, then a final division by N
 *     (Sec. IV, iNTT paragraph).
 *   - HE Mul flow: Fig. 2 (region 1 tensor, region 2 key switching with evk,
 *     shift), rescale by division (Sec. III-A).
 *   - Full-RNS form (mod up / mod down): Table XI and the Discussion section
 *     (its part on other libraries); the paper only names these
 *     functions, so the formulas below are the standard fast base conversion
 *     of full-RNS CKKS: non-centred sources, no overflow correction, mod down
 *     without a rounding offset, rescale rounding to nearest by the centred
 *     lift of the dropped limb.
 *
 * Parity status: NTT/INTT pinned (closed form, schoolbook convolution,
 * round trip); ModUp, ModDown, rescale pinned by big-integer identities at
 * tiny N; key generation/encryption take all random draws as inputs.
 *
 * Optional OpenMP over limbs only shortens wall time; it does not change
 * any arithmetic or its order within a limb.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops over limbs (timing only; results do not
 * depend on it).  Returns the count the runtime will use. */
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

typedef unsigned __int128 u128;

/* ---------- scalar modular arithmetic (plain definitions) ---------- */
static uint64_t mmul(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)(((u128)a * b) % m); }
static uint64_t madd(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)(((u128)a + b) % m); }
static uint64_t msub(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)(((u128)a + m - b) % m); }
static uint64_t mpow(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m; a %= m;
  while (e) { if (e & 1) r = mmul(r, a, m); a = mmul(a, a, m); e >>= 1; }
  return r;
}
/* inverse by Fermat's little theorem (m prime) */
static uint64_t minv(uint64_t a, uint64_t m) { return mpow(a, m - 2, m); }
/* signed integer -> canonical residue */
static uint64_t mfrom_i64(int64_t x, uint64_t m) {
  int64_t r = (int64_t)((x % (int64_t)m + (int64_t)m) % (int64_t)m);
  return (uint64_t)r;
}

/* Counters for the operation-count pin (Table IV): modular multiplications
 * performed inside NTT and iNTT. */
static uint64_t g_ntt_modmul = 0, g_intt_modmul = 0;
uint64_t orc_counter_ntt(void) { return g_ntt_modmul; }
uint64_t orc_counter_intt(void) { return g_intt_modmul; }
void orc_counter_reset(void) { g_ntt_modmul = 0; g_intt_modmul = 0; }

/* ---------- primes ---------- */
/* Deterministic Miller-Rabin for n < 2^64 (first twelve prime bases). */
int orc_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) { if (n % bases[i] == 0) return n == bases[i]; }
  uint64_t d = n - 1; int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = mpow(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int r = 1; r < s; ++r) { x = mmul(x, x, n); if (x == n - 1) { comp = 0; break; } }
    if (comp) return 0;
  }
  return 1;
}

/* The `count` largest primes x < 2^bits with x = 1 (mod 2N), scanned
 * downward, skipping any listed in `exclude`.  Returns number found. */
int orc_gen_primes(uint32_t log_n, uint32_t bits, uint32_t count, const uint64_t* exclude,
                   uint32_t nexclude, uint64_t* out) {
  uint64_t twoN = 2ull << log_n;
  uint64_t x = ((1ull << bits) - 1) / twoN * twoN + 1; /* largest 1 mod 2N below 2^bits */
  if (x >= (1ull << bits)) x -= twoN;
  uint32_t found = 0;
  while (found < count && x > twoN) {
    if (orc_is_prime(x)) {
      int ex = 0;
      for (uint32_t i = 0; i < nexclude; ++i) if (exclude[i] == x) ex = 1;
      if (!ex) out[found++] = x;
    }
    x -= twoN;
  }
  return (int)found;
}

/* The smallest primitive 2N-th root of unity modulo prime q (q = 1 mod 2N).
 * Any x with x^N = -1 is primitive of order 2N; all such roots are its odd
 * powers.  Returns 0 if q is not 1 mod 2N. */
uint64_t orc_min_root(uint64_t q, uint32_t log_n) {
  uint64_t N = 1ull << log_n, twoN = 2 * N;
  if ((q - 1) % twoN != 0) return 0;
  uint64_t g = 0;
  for (uint64_t c = 2; c < q; ++c) {
    uint64_t r = mpow(c, (q - 1) / twoN, q);
    if (mpow(r, N, q) == q - 1) { g = r; break; }
  }
  uint64_t best = g, r2 = mmul(g, g, q), cur = g;
  for (uint64_t k = 3; k < twoN; k += 2) { cur = mmul(cur, r2, q); if (cur < best) best = cur; }
  return best;
}

/* ---------- negacyclic NTT by recursive factorisation ---------- */
/* The forward transform evaluates a in Z_q[X]/(X^N + 1) at the N roots of
 * X^N + 1, which are the odd powers of psi (Sec. IV, NTT: the negacyclic
 * transform with the 2N-th root merged in).  It is written here as the
 * Chinese-remainder split of the modulus polynomial rather than as a loop
 * nest.  Write the modulus of a node of n coefficients as X^n - psi^E.  With
 * s = psi^(E/2) it factors as (X^(n/2) - s)(X^(n/2) + s), and for
 * a = lo + X^(n/2) hi
 *     a mod (X^(n/2) - s) = lo + s hi,      a mod (X^(n/2) + s) = lo - s hi,
 * where X^(n/2) + s = X^(n/2) - psi^(E/2 + N) because psi^N = -1.  The root
 * node is X^N + 1 = X^N - psi^N; a leaf (n = 1) holds a mod (X - psi^E) =
 * a(psi^E).  Placing the first factor's residue in the first half and the
 * second's in the second half leaves a(psi^(2 brv(i) + 1)) at position i
 * (bit-reversed order).  One modular product per coefficient pair and
 * level: N/2 log N in all, the count of Table IV.
 * pw[k] = psi^k mod q for 0 <= k < 2N. */
static void ntt_split(uint64_t* a, uint64_t n, uint64_t E, uint64_t q, const uint64_t* pw, uint64_t N) {
  if (n < 2) return;
  uint64_t h = n / 2, s = pw[E / 2];
  for (uint64_t k = 0; k < h; ++k) {
    uint64_t t = mmul(s, a[h + k], q);
    g_ntt_modmul++;
    uint64_t lo = a[k];
    a[k] = madd(lo, t, q);
    a[h + k] = msub(lo, t, q);
  }
  ntt_split(a, h, E / 2, q, pw, N);
  ntt_split(a + h, h, E / 2 + N, q, pw, N);
}
/* The inverse undoes each split from the leaves up: from u = lo + s hi and
 * v = lo - s hi it forms u + v = 2 lo and (u - v) s^(-1) = 2 hi, with
 * s^(-1) = psi^(2N - E/2).  Every level doubles the values, so the result
 * is N a, and a final product by N^(-1) gives a: N/2 log N + N modular
 * products, the iNTT count of Table IV. */
static void intt_split(uint64_t* a, uint64_t n, uint64_t E, uint64_t q, const uint64_t* pw, uint64_t N) {
  if (n < 2) return;
  uint64_t h = n / 2, sinv = pw[2 * N - E / 2];
  intt_split(a, h, E / 2, q, pw, N);
  intt_split(a + h, h, E / 2 + N, q, pw, N);
  for (uint64_t k = 0; k < h; ++k) {
    uint64_t u = a[k], v = a[h + k];
    a[k] = madd(u, v, q);
    a[h + k] = mmul(msub(u, v, q), sinv, q);
    g_intt_modmul++;
  }
}
static void ntt_core(uint64_t* a, uint32_t log_n, uint64_t q, const uint64_t* pw) {
  uint64_t N = 1ull << log_n;
  ntt_split(a, N, N, q, pw, N);
}
static void intt_core(uint64_t* a, uint32_t log_n, uint64_t q, const uint64_t* pw) {
  uint64_t N = 1ull << log_n;
  intt_split(a, N, N, q, pw, N);
  uint64_t ninv = minv(N % q, q);
  for (uint64_t i = 0; i < N; ++i) { a[i] = mmul(a[i], ninv, q); g_intt_modmul++; }
}

/* ---------- context: moduli and tables ---------- */
typedef struct {
  uint32_t log_n, L, K, dnum, alpha;
  uint64_t N;
  uint64_t* mod;    /* [L+K]: q_0..q_{L-1}, p_0..p_{K-1} */
  uint64_t* psi;    /* [L+K] */
  uint64_t* pw;     /* [L+K][2N]: psi^k, 0 <= k < 2N */
} orc_ctx;

orc_ctx* orc_ctx_new(uint32_t log_n, uint32_t L, uint32_t K, uint32_t dnum, const uint64_t* q,
                     const uint64_t* p) {
  orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  c->log_n = log_n; c->L = L; c->K = K; c->dnum = dnum; c->N = 1ull << log_n;
  c->alpha = (L + dnum - 1) / dnum;
  uint32_t nm = L + K;
  c->mod = (uint64_t*)malloc(sizeof(uint64_t) * nm);
  for (uint32_t i = 0; i < L; ++i) c->mod[i] = q[i];
  for (uint32_t k = 0; k < K; ++k) c->mod[L + k] = p[k];
  c->psi = (uint64_t*)malloc(sizeof(uint64_t) * nm);
  c->pw = (uint64_t*)malloc(sizeof(uint64_t) * nm * 2 * c->N);
#pragma omp parallel for schedule(dynamic)
  for (uint32_t i = 0; i < nm; ++i) {
    uint64_t m = c->mod[i];
    uint64_t psi = orc_min_root(m, log_n);
    uint64_t* pw = c->pw + (uint64_t)i * 2 * c->N;
    c->psi[i] = psi;
    pw[0] = 1 % m;
    for (uint64_t k = 1; k < 2 * c->N; ++k) pw[k] = mmul(pw[k - 1], psi, m);
  }
  return c;
}
void orc_ctx_free(orc_ctx* c) {
  if (!c) return;
  free(c->mod); free(c->psi); free(c->pw); free(c);
}
uint64_t orc_psi(const orc_ctx* c, uint32_t idx) { return c->psi[idx]; }
const uint64_t* orc_powers(const orc_ctx* c, uint32_t idx) { return c->pw + (uint64_t)idx * 2 * c->N; }

/* NTT / INTT of one limb modulo basis element `idx` (0..L+K-1). */
void orc_ntt(const orc_ctx* c, uint32_t idx, uint64_t* a) {
  ntt_core(a, c->log_n, c->mod[idx], c->pw + (uint64_t)idx * 2 * c->N);
}
void orc_intt(const orc_ctx* c, uint32_t idx, uint64_t* a) {
  intt_core(a, c->log_n, c->mod[idx], c->pw + (uint64_t)idx * 2 * c->N);
}

/* basis position e of the extended basis E_l = {q_0..q_{l-1}, p_0..p_{K-1}}
 * -> index into c->mod */
static uint32_t ext_idx(const orc_ctx* c, uint32_t level, uint32_t e) {
  return e < level ? e : c->L + (e - level);
}

/* ---------- region 1: tensor product (Fig. 2) ---------- */
/* ct = [2][level][N], poly 0 = b (bx), poly 1 = a (ax), NTT form.
 * d = [3][level][N]: d0 = b1 b2, d1 = a1 b2 + a2 b1, d2 = a1 a2. */
void orc_tensor(const orc_ctx* c, uint32_t level, const uint64_t* ct1, const uint64_t* ct2,
                uint64_t* d) {
  uint64_t N = c->N, P = (uint64_t)level * N;
  for (uint32_t i = 0; i < level; ++i) {
    uint64_t q = c->mod[i];
    for (uint64_t k = 0; k < N; ++k) {
      uint64_t o = (uint64_t)i * N + k;
      uint64_t b1 = ct1[o], a1 = ct1[P + o], b2 = ct2[o], a2 = ct2[P + o];
      d[o] = mmul(b1, b2, q);
      d[P + o] = madd(mmul(a1, b2, q), mmul(a2, b1, q), q);
      d[2 * P + o] = mmul(a1, a2, q);
    }
  }
}

/* number of nonempty digits at level l */
uint32_t orc_num_digits(const orc_ctx* c, uint32_t level) { return (level + c->alpha - 1) / c->alpha; }

/* ---------- ModUp (fast base conversion, one digit) ---------- */
/* d2: [level][N] NTT form.  dt: [beta][level+K][N] NTT form (dt_j over E_l). */
void orc_modup(const orc_ctx* c, uint32_t level, const uint64_t* d2, uint64_t* dt) {
  uint64_t N = c->N;
  uint32_t beta = orc_num_digits(c, level), ne = level + c->K;
  uint64_t* x = (uint64_t*)malloc(sizeof(uint64_t) * level * N);
  memcpy(x, d2, sizeof(uint64_t) * level * N);
#pragma omp parallel for schedule(dynamic)
  for (uint32_t i = 0; i < level; ++i) orc_intt(c, i, x + (uint64_t)i * N);
  for (uint32_t j = 0; j < beta; ++j) {
    uint32_t lo = j * c->alpha, hi = (j + 1) * c->alpha < level ? (j + 1) * c->alpha : level;
    uint64_t* out = dt + (uint64_t)j * ne * N;
    /* y_i = x_i * [(Qt_j / q_i)^{-1}]_{q_i}, i in D_j */
    uint64_t* y = (uint64_t*)malloc(sizeof(uint64_t) * (hi - lo) * N);
    for (uint32_t i = lo; i < hi; ++i) {
      uint64_t qi = c->mod[i], prod = 1 % qi;
      for (uint32_t i2 = lo; i2 < hi; ++i2) if (i2 != i) prod = mmul(prod, c->mod[i2] % qi, qi);
      uint64_t inv = minv(prod, qi);
      for (uint64_t k = 0; k < N; ++k) y[(uint64_t)(i - lo) * N + k] = mmul(x[(uint64_t)i * N + k], inv, qi);
    }
#pragma omp parallel for schedule(dynamic)
    for (uint32_t e = 0; e < ne; ++e) {
      uint64_t* dst = out + (uint64_t)e * N;
      if (e >= lo && e < hi) { /* own limbs: the NTT-form input itself */
        memcpy(dst, d2 + (uint64_t)e * N, sizeof(uint64_t) * N);
        continue;
      }
      uint64_t t = c->mod[ext_idx(c, level, e)];
      /* [Qt_j / q_i]_t for each i in D_j */
      uint64_t* hat = (uint64_t*)malloc(sizeof(uint64_t) * (hi - lo));
      for (uint32_t i = lo; i < hi; ++i) {
        uint64_t prod = 1 % t;
        for (uint32_t i2 = lo; i2 < hi; ++i2) if (i2 != i) prod = mmul(prod, c->mod[i2] % t, t);
        hat[i - lo] = prod;
      }
      for (uint64_t k = 0; k < N; ++k) {
        uint64_t z = 0;
        for (uint32_t i = lo; i < hi; ++i) z = madd(z, mmul(y[(uint64_t)(i - lo) * N + k] % t, hat[i - lo], t), t);
        dst[k] = z;
      }
      free(hat);
      orc_ntt(c, ext_idx(c, level, e), dst);
    }
    free(y);
  }
  free(x);
}

/* ---------- inner product with evk (region 2) ---------- */
/* evk: [dnum][2][L+K][N] NTT form, poly 0 = b, poly 1 = a.
 * ks: [2][level+K][N]: ks_u[e] = sum_j dt_j[e] * evk_j.u[e] */
void orc_inner_product(const orc_ctx* c, uint32_t level, const uint64_t* dt, const uint64_t* evk,
                       uint64_t* ks) {
  uint64_t N = c->N;
  uint32_t beta = orc_num_digits(c, level), ne = level + c->K, nm = c->L + c->K;
#pragma omp parallel for schedule(dynamic)
  for (uint32_t e = 0; e < ne; ++e) {
    uint32_t mi = ext_idx(c, level, e);
    uint64_t m = c->mod[mi];
    for (uint32_t u = 0; u < 2; ++u) {
      for (uint64_t k = 0; k < N; ++k) {
        uint64_t acc = 0;
        for (uint32_t j = 0; j < beta; ++j) {
          uint64_t dv = dt[((uint64_t)j * ne + e) * N + k];
          uint64_t ev = evk[(((uint64_t)j * 2 + u) * nm + mi) * N + k];
          acc = madd(acc, mmul(dv, ev, m), m);
        }
        ks[((uint64_t)u * ne + e) * N + k] = acc;
      }
    }
  }
}

/* ---------- ModDown + combine ---------- */
/* ks: [2][level+K][N] NTT; d: [3][level][N] tensor output.
 * out: [2][level][N] NTT: b' = d0 + moddown(ks_b), a' = d1 + moddown(ks_a). */
void orc_moddown_combine(const orc_ctx* c, uint32_t level, const uint64_t* ks, const uint64_t* d,
                         uint64_t* out) {
  uint64_t N = c->N;
  uint32_t K = c->K, ne = level + K;
  /* constants */
  uint64_t* phat_inv = (uint64_t*)malloc(sizeof(uint64_t) * K);       /* [(P/p_k)^{-1}]_{p_k} */
  uint64_t* phat_q = (uint64_t*)malloc(sizeof(uint64_t) * K * level); /* [P/p_k]_{q_i} */
  uint64_t* pinv_q = (uint64_t*)malloc(sizeof(uint64_t) * level);     /* [P^{-1}]_{q_i} */
  for (uint32_t k = 0; k < K; ++k) {
    uint64_t pk = c->mod[c->L + k], prod = 1 % pk;
    for (uint32_t k2 = 0; k2 < K; ++k2) if (k2 != k) prod = mmul(prod, c->mod[c->L + k2] % pk, pk);
    phat_inv[k] = minv(prod, pk);
    for (uint32_t i = 0; i < level; ++i) {
      uint64_t qi = c->mod[i], pr = 1 % qi;
      for (uint32_t k2 = 0; k2 < K; ++k2) if (k2 != k) pr = mmul(pr, c->mod[c->L + k2] % qi, qi);
      phat_q[(uint64_t)k * level + i] = pr;
    }
  }
  for (uint32_t i = 0; i < level; ++i) {
    uint64_t qi = c->mod[i], pr = 1 % qi;
    for (uint32_t k = 0; k < K; ++k) pr = mmul(pr, c->mod[c->L + k] % qi, qi);
    pinv_q[i] = minv(pr, qi);
  }
  uint64_t* y = (uint64_t*)malloc(sizeof(uint64_t) * K * N);
  for (uint32_t u = 0; u < 2; ++u) {
    const uint64_t* ksu = ks + (uint64_t)u * ne * N;
#pragma omp parallel for schedule(dynamic)
    for (uint32_t k = 0; k < K; ++k) {
      uint64_t pk = c->mod[c->L + k];
      uint64_t* yk = y + (uint64_t)k * N;
      memcpy(yk, ksu + (uint64_t)(level + k) * N, sizeof(uint64_t) * N);
      orc_intt(c, c->L + k, yk);
      for (uint64_t n = 0; n < N; ++n) yk[n] = mmul(yk[n], phat_inv[k], pk);
    }
#pragma omp parallel for schedule(dynamic)
    for (uint32_t i = 0; i < level; ++i) {
      uint64_t qi = c->mod[i];
      uint64_t* z = (uint64_t*)malloc(sizeof(uint64_t) * N);
      for (uint64_t n = 0; n < N; ++n) {
        uint64_t acc = 0;
        for (uint32_t k = 0; k < K; ++k)
          acc = madd(acc, mmul(y[(uint64_t)k * N + n] % qi, phat_q[(uint64_t)k * level + i], qi), qi);
        z[n] = acc;
      }
      orc_ntt(c, i, z);
      const uint64_t* dd = d + ((uint64_t)u * level + i) * N;
      uint64_t* o = out + ((uint64_t)u * level + i) * N;
      for (uint64_t n = 0; n < N; ++n) {
        uint64_t md = mmul(msub(ksu[(uint64_t)i * N + n], z[n], qi), pinv_q[i], qi);
        o[n] = madd(dd[n], md, qi);
      }
      free(z);
    }
  }
  free(y); free(phat_inv); free(phat_q); free(pinv_q);
}

/* ---------- rescale (Sec. III-A: divide by the last prime) ---------- */
/* in: [2][level][N] NTT; out: [2][level-1][N] NTT. */
void orc_rescale(const orc_ctx* c, uint32_t level, const uint64_t* in, uint64_t* out) {
  uint64_t N = c->N;
  uint32_t last = level - 1;
  uint64_t ql = c->mod[last];
  uint64_t* r = (uint64_t*)malloc(sizeof(uint64_t) * N);
  for (uint32_t u = 0; u < 2; ++u) {
    memcpy(r, in + ((uint64_t)u * level + last) * N, sizeof(uint64_t) * N);
    orc_intt(c, last, r);
#pragma omp parallel for schedule(dynamic)
    for (uint32_t i = 0; i < last; ++i) {
      uint64_t qi = c->mod[i];
      uint64_t qlinv = minv(ql % qi, qi);
      uint64_t* s = (uint64_t*)malloc(sizeof(uint64_t) * N);
      for (uint64_t n = 0; n < N; ++n) {
        /* centered representative r^c in (-ql/2, ql/2), reduced into [0, qi) */
        if (2 * (u128)r[n] < ql) s[n] = r[n] % qi;
        else s[n] = msub(r[n] % qi, ql % qi, qi);
      }
      orc_ntt(c, i, s);
      const uint64_t* ci = in + ((uint64_t)u * level + i) * N;
      uint64_t* o = out + ((uint64_t)u * last + i) * N;
      for (uint64_t n = 0; n < N; ++n) o[n] = mmul(msub(ci[n], s[n], qi), qlinv, qi);
      free(s);
    }
  }
  free(r);
}

/* ---------- whole HE Mul ---------- */
/* relin: [2][level][N] (after key switching, before rescale), may be NULL.
 * out: [2][level-1][N] (after rescale), may be NULL. */
void orc_he_mul(const orc_ctx* c, uint32_t level, const uint64_t* ct1, const uint64_t* ct2,
                const uint64_t* evk, uint64_t* relin, uint64_t* out) {
  uint64_t N = c->N;
  uint32_t beta = orc_num_digits(c, level), ne = level + c->K;
  uint64_t* d = (uint64_t*)malloc(sizeof(uint64_t) * 3 * level * N);
  uint64_t* dt = (uint64_t*)malloc(sizeof(uint64_t) * (uint64_t)beta * ne * N);
  uint64_t* ks = (uint64_t*)malloc(sizeof(uint64_t) * 2 * ne * N);
  uint64_t* rl = (uint64_t*)malloc(sizeof(uint64_t) * 2 * level * N);
  orc_tensor(c, level, ct1, ct2, d);
  orc_modup(c, level, d + 2ull * level * N, dt);
  orc_inner_product(c, level, dt, evk, ks);
  orc_moddown_combine(c, level, ks, d, rl);
  if (relin) memcpy(relin, rl, sizeof(uint64_t) * 2 * level * N);
  if (out && level >= 2) orc_rescale(c, level, rl, out);
  free(d); free(dt); free(ks); free(rl);
}

/* ---------- keys and encryption (all random draws are inputs) ---------- */
/* Signed small polynomial -> NTT form limb for basis index idx. */
static void small_to_ntt(const orc_ctx* c, uint32_t idx, const int64_t* v, uint64_t* dst) {
  uint64_t m = c->mod[idx];
  for (uint64_t n = 0; n < c->N; ++n) dst[n] = mfrom_i64(v[n], m);
  orc_ntt(c, idx, dst);
}

/* Public key over q_0..q_{L-1}: b = a*s + e, a uniform (given, NTT form).
 * a_unif: [L][N]; pk: [2][L][N]. */
void orc_keygen_pk(const orc_ctx* c, const int64_t* s, const int64_t* e, const uint64_t* a_unif,
                   uint64_t* pk) {
  uint64_t N = c->N;
  uint32_t L = c->L;
#pragma omp parallel for schedule(dynamic)
  for (uint32_t i = 0; i < L; ++i) {
    uint64_t m = c->mod[i];
    uint64_t* sn = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* en = (uint64_t*)malloc(sizeof(uint64_t) * N);
    small_to_ntt(c, i, s, sn);
    small_to_ntt(c, i, e, en);
    for (uint64_t n = 0; n < N; ++n) {
      uint64_t a = a_unif[(uint64_t)i * N + n];
      pk[(uint64_t)i * N + n] = madd(mmul(a, sn[n], m), en[n], m);
      pk[((uint64_t)L + i) * N + n] = a;
    }
    free(sn); free(en);
  }
}

/* Evaluation key (hybrid gadget, dnum digits) over q_0..q_{L-1}, p_0..p_{K-1}:
 * b_j = a_j*s + e_j + G_j*s^2 with G_j = [P]_{q_i} for i in digit j, 0 on
 * other q_i and on every p_k.  a_unif: [dnum][L+K][N]; e: [dnum][N];
 * evk: [dnum][2][L+K][N]. */
void orc_keygen_evk(const orc_ctx* c, const int64_t* s, const int64_t* e, const uint64_t* a_unif,
                    uint64_t* evk) {
  uint64_t N = c->N;
  uint32_t L = c->L, K = c->K, nm = L + K;
#pragma omp parallel for schedule(dynamic)
  for (uint32_t i = 0; i < nm; ++i) {
    uint64_t m = c->mod[i];
    uint64_t Pm = 1 % m;
    for (uint32_t k = 0; k < K; ++k) Pm = mmul(Pm, c->mod[L + k] % m, m);
    uint64_t* sn = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* en = (uint64_t*)malloc(sizeof(uint64_t) * N);
    small_to_ntt(c, i, s, sn);
    for (uint32_t j = 0; j < c->dnum; ++j) {
      small_to_ntt(c, i, e + (uint64_t)j * N, en);
      int in_digit = (i < L) && (i / c->alpha == j);
      for (uint64_t n = 0; n < N; ++n) {
        uint64_t a = a_unif[((uint64_t)j * nm + i) * N + n];
        uint64_t b = madd(mmul(a, sn[n], m), en[n], m);
        if (in_digit) b = madd(b, mmul(Pm, mmul(sn[n], sn[n], m), m), m);
        evk[(((uint64_t)j * 2 + 0) * nm + i) * N + n] = b;
        evk[(((uint64_t)j * 2 + 1) * nm + i) * N + n] = a;
      }
    }
    free(sn); free(en);
  }
}

/* ct = (v*pk.b + e0 + m, v*pk.a + e1) at `level`, NTT form.  m, v, e0, e1
 * are signed coefficient vectors of length N.  pk: [2][L][N]. */
void orc_encrypt(const orc_ctx* c, uint32_t level, const int64_t* msg, const int64_t* v,
                 const int64_t* e0, const int64_t* e1, const uint64_t* pk, uint64_t* ct) {
  uint64_t N = c->N;
  uint32_t L = c->L;
#pragma omp parallel for schedule(dynamic)
  for (uint32_t i = 0; i < level; ++i) {
    uint64_t q = c->mod[i];
    uint64_t* vn = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* t0 = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* t1 = (uint64_t*)malloc(sizeof(uint64_t) * N);
    small_to_ntt(c, i, v, vn);
    for (uint64_t n = 0; n < N; ++n) t0[n] = madd(mfrom_i64(e0[n], q), mfrom_i64(msg[n], q), q);
    orc_ntt(c, i, t0);
    small_to_ntt(c, i, e1, t1);
    for (uint64_t n = 0; n < N; ++n) {
      ct[(uint64_t)i * N + n] = madd(mmul(vn[n], pk[(uint64_t)i * N + n], q), t0[n], q);
      ct[((uint64_t)level + i) * N + n] = madd(mmul(vn[n], pk[((uint64_t)L + i) * N + n], q), t1[n], q);
    }
    free(vn); free(t0); free(t1);
  }
}

/* m = INTT(b - a*s) per limb: [level][N] coefficient residues. */
void orc_decrypt_limbs(const orc_ctx* c, uint32_t level, const uint64_t* ct, const int64_t* s,
                       uint64_t* m_out) {
  uint64_t N = c->N;
#pragma omp parallel for schedule(dynamic)
  for (uint32_t i = 0; i < level; ++i) {
    uint64_t q = c->mod[i];
    uint64_t* sn = (uint64_t*)malloc(sizeof(uint64_t) * N);
    small_to_ntt(c, i, s, sn);
    uint64_t* o = m_out + (uint64_t)i * N;
    for (uint64_t n = 0; n < N; ++n)
      o[n] = msub(ct[(uint64_t)i * N + n], mmul(ct[((uint64_t)level + i) * N + n], sn[n], q), q);
    orc_intt(c, i, o);
    free(sn);
  }
}

/* ---------- rotation: automorphism X -> X^g and key switching ---------- */
/* The automorphism of a polynomial in coefficient form, by its definition:
 * the term a_k X^k goes to a_k X^(k g mod 2N), negated when k g mod 2N >= N
 * (X^N = -1).  g odd.  in, out: [N] residues mod m (out != in). */
static void automorphism_coeff(const uint64_t* in, uint64_t* out, uint64_t N, uint64_t g, uint64_t m) {
  for (uint64_t k = 0; k < N; ++k) {
    uint64_t e = (uint64_t)(((u128)k * g) % (2 * N));
    if (e < N) out[e] = in[k];
    else out[e - N] = in[k] ? m - in[k] : 0;
  }
}

/* sigma_g of a ciphertext [2][level][N] in NTT form: INTT, the automorphism
 * in coefficient form, NTT. */
void orc_automorphism(const orc_ctx* c, uint32_t level, uint64_t g, const uint64_t* in, uint64_t* out) {
  uint64_t N = c->N;
#pragma omp parallel for schedule(dynamic)
  for (uint32_t t = 0; t < 2 * level; ++t) {
    uint32_t i = t % level;
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * N);
    memcpy(tmp, in + (uint64_t)t * N, sizeof(uint64_t) * N);
    orc_intt(c, i, tmp);
    automorphism_coeff(tmp, out + (uint64_t)t * N, N, g, c->mod[i]);
    orc_ntt(c, i, out + (uint64_t)t * N);
    free(tmp);
  }
}

/* Rotation key for sigma_g: the evaluation key of the secret -sigma_g(s)
 * in place of s^2 (b_j = a_j s + e_j - G_j sigma_g(s)), so that key
 * switching sigma_g(a) gives a pair decrypting, under s, to
 * -sigma_g(a) sigma_g(s).  Same layout as the evaluation key. */
void orc_keygen_rot(const orc_ctx* c, const int64_t* s, uint64_t g, const int64_t* e, const uint64_t* a_unif,
                    uint64_t* rk) {
  uint64_t N = c->N;
  uint32_t L = c->L, K = c->K, nm = L + K;
  int64_t* sg = (int64_t*)malloc(sizeof(int64_t) * N);  /* -sigma_g(s) as a signed polynomial */
  for (uint64_t k = 0; k < N; ++k) {
    uint64_t ex = (uint64_t)(((u128)k * g) % (2 * N));
    if (ex < N) sg[ex] = -s[k];
    else sg[ex - N] = s[k];
  }
#pragma omp parallel for schedule(dynamic)
  for (uint32_t i = 0; i < nm; ++i) {
    uint64_t m = c->mod[i];
    uint64_t Pm = 1 % m;
    for (uint32_t k = 0; k < K; ++k) Pm = mmul(Pm, c->mod[L + k] % m, m);
    uint64_t* sn = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* gn = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* en = (uint64_t*)malloc(sizeof(uint64_t) * N);
    small_to_ntt(c, i, s, sn);
    small_to_ntt(c, i, sg, gn);
    for (uint32_t j = 0; j < c->dnum; ++j) {
      small_to_ntt(c, i, e + (uint64_t)j * N, en);
      int in_digit = (i < L) && (i / c->alpha == j);
      for (uint64_t n = 0; n < N; ++n) {
        uint64_t a = a_unif[((uint64_t)j * nm + i) * N + n];
        uint64_t b = madd(mmul(a, sn[n], m), en[n], m);
        if (in_digit) b = madd(b, mmul(Pm, gn[n], m), m);
        rk[(((uint64_t)j * 2 + 0) * nm + i) * N + n] = b;
        rk[(((uint64_t)j * 2 + 1) * nm + i) * N + n] = a;
      }
    }
    free(sn); free(gn); free(en);
  }
  free(sg);
}

/* Rotation of a ciphertext [2][level][N] (NTT form): (sigma_g(b), sigma_g(a))
 * key-switched back to s with rk: out = (sigma_g(b) + KS_b, KS_a), where KS
 * is ModUp, inner product with rk and ModDown of sigma_g(a) (the triple
 * (sigma_g(b), 0, sigma_g(a)) through the same steps as HE Mul). */
void orc_rotate(const orc_ctx* c, uint32_t level, uint64_t g, const uint64_t* ct, const uint64_t* rk,
                uint64_t* out) {
  uint64_t N = c->N;
  uint32_t beta = orc_num_digits(c, level), ne = level + c->K;
  uint64_t* sct = (uint64_t*)malloc(sizeof(uint64_t) * 2 * level * N);
  uint64_t* d = (uint64_t*)calloc(3 * (uint64_t)level * N, sizeof(uint64_t));
  uint64_t* dt = (uint64_t*)malloc(sizeof(uint64_t) * (uint64_t)beta * ne * N);
  uint64_t* ks = (uint64_t*)malloc(sizeof(uint64_t) * 2 * ne * N);
  orc_automorphism(c, level, g, ct, sct);
  memcpy(d, sct, sizeof(uint64_t) * level * N);                               /* d0 = sigma(b) */
  memcpy(d + 2ull * level * N, sct + (uint64_t)level * N, sizeof(uint64_t) * level * N); /* d2 = sigma(a) */
  orc_modup(c, level, d + 2ull * level * N, dt);
  orc_inner_product(c, level, dt, rk, ks);
  orc_moddown_combine(c, level, ks, d, out);
  free(sct); free(d); free(dt); free(ks);
}
