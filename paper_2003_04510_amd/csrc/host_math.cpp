#include "host_math.hpp"

namespace he {

u64 powmod(u64 a, u64 e, u64 m) {
  u64 r = 1 % m;
  a %= m;
  for (; e; e >>= 1) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
  }
  return r;
}

namespace {

// Jacobi symbol (a / n) for odd n > 0, by the binary reciprocity algorithm.
int jacobi(u64 a, u64 n) {
  a %= n;
  int t = 1;
  while (a) {
    while (!(a & 1)) {
      a >>= 1;
      const u64 r = n & 7;
      if (r == 3 || r == 5) t = -t;
    }
    const u64 tmp = a;
    a = n;
    n = tmp;
    if ((a & 3) == 3 && (n & 3) == 3) t = -t;
    a %= n;
  }
  return n == 1 ? t : 0;
}

// Jacobi symbol (d / n) for a signed d.
int jacobi_signed(int64_t d, u64 n) {
  if (d >= 0) return jacobi((u64)d, n);
  const int j = jacobi((u64)(-d), n);
  return (n & 3) == 3 ? -j : j;  // (-1 / n) = -1 iff n = 3 mod 4
}

bool is_square(u64 n) {
  u64 r = (u64)__builtin_sqrtl((long double)n);
  while (r * r > n) --r;
  while ((r + 1) * (r + 1) <= n) ++r;
  return r * r == n;
}

// Strong probable prime to base 2 (n odd, n > 2).
bool strong_base2(u64 n) {
  u64 d = n - 1;
  const int s = __builtin_ctzll(d);
  d >>= s;
  u64 x = powmod(2, d, n);
  if (x == 1 || x == n - 1) return true;
  for (int r = 1; r < s; ++r) {
    x = mulmod(x, x, n);
    if (x == n - 1) return true;
  }
  return false;
}

// x / 2 mod n for odd n
u64 half(u64 x, u64 n) { return (x & 1) ? (u64)(((u128)x + n) >> 1) : x >> 1; }

// Strong Lucas probable prime with Selfridge's parameters: D the first of
// 5, -7, 9, -11, ... with (D / n) = -1, P = 1, Q = (1 - D) / 4 (n odd, not a
// square).
bool strong_lucas(u64 n) {
  int64_t D = 5;
  for (;;) {
    const int j = jacobi_signed(D, n);
    if (j == -1) break;
    if (j == 0 && (u64)(D < 0 ? -D : D) != n) return false;  // a factor of n
    D = D > 0 ? -(D + 2) : -D + 2;
  }
  const u64 Dm = D >= 0 ? (u64)D % n : n - ((u64)(-D) % n);
  const int64_t Qs = (1 - D) / 4;
  const u64 Qm = Qs >= 0 ? (u64)Qs % n : n - ((u64)(-Qs) % n);
  // n + 1 = d 2^s, d odd
  u64 d = n + 1;
  const int s = __builtin_ctzll(d);
  d >>= s;
  // U_k, V_k, Q^k for k = the leading bits of d, from the top bit down
  u64 U = 1, V = 1, Qk = Qm;  // k = 1: U_1 = 1, V_1 = P = 1
  for (int b = 62 - __builtin_clzll(d); b >= 0; --b) {
    // doubling: U_2k = U_k V_k, V_2k = V_k^2 - 2 Q^k, Q^2k = (Q^k)^2
    U = mulmod(U, V, n);
    V = submod(mulmod(V, V, n), addmod(Qk, Qk, n), n);
    Qk = mulmod(Qk, Qk, n);
    if ((d >> b) & 1) {
      // k -> k + 1 (P = 1): U' = (U + V) / 2, V' = (D U + V) / 2
      const u64 U1 = half(addmod(U, V, n), n);
      const u64 V1 = half(addmod(mulmod(Dm, U, n), V, n), n);
      U = U1;
      V = V1;
      Qk = mulmod(Qk, Qm, n);
    }
  }
  if (U == 0 || V == 0) return true;
  for (int r = 1; r < s; ++r) {
    V = submod(mulmod(V, V, n), addmod(Qk, Qk, n), n);
    Qk = mulmod(Qk, Qk, n);
    if (V == 0) return true;
  }
  return false;
}

}  // namespace

// Baillie-PSW: trial division by small primes, a strong probable-prime test
// to base 2 and a strong Lucas test.  No composite below 2^64 passes both
// (checked against the complete list of base-2 strong pseudoprimes below
// 2^64), so the test is exact for 64-bit n.
bool is_prime(u64 n) {
  static const unsigned small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71};
  if (n < 2) return false;
  for (unsigned p : small) {
    if (n == p) return true;
    if (n % p == 0) return false;
  }
  if (n < 73 * 73) return true;
  if (!strong_base2(n)) return false;
  if (is_square(n)) return false;
  return strong_lucas(n);
}

// Candidates 1 mod 2N below 2^bits are k 2N + 1; k runs downward from the
// largest one below the bound.
bool gen_primes(unsigned log_n, unsigned bits, unsigned count, const u64* excl, unsigned nexcl,
                u64* out) {
  const u64 step = 2ull << log_n;
  const u64 bound = bits >= 64 ? ~0ull : (1ull << bits);  // exclusive (inclusive for 64)
  unsigned found = 0;
  for (u64 k = (bound - 2) / step; k >= 1 && found < count; --k) {
    const u64 x = k * step + 1;
    bool listed = false;
    for (unsigned i = 0; i < nexcl && !listed; ++i) listed = excl[i] == x;
    if (!listed && is_prime(x)) out[found++] = x;
  }
  return found == count;
}

// A quadratic non-residue c (Jacobi symbol -1) generates the whole 2-Sylow
// subgroup of (Z/mZ)*: with m - 1 = 2^e t, t odd, c^t has order 2^e, so
// g = c^((m-1)/2N) has order exactly 2N.  The primitive 2N-th roots are the
// odd powers of g; the smallest of them is returned.
u64 min_root_2n(u64 m, unsigned log_n) {
  const u64 two_n = 2ull << log_n;
  if ((m - 1) % two_n) return 0;
  u64 c = 2;
  while (jacobi(c, m) != -1) ++c;
  const u64 g = powmod(c, (m - 1) / two_n, m);
  const u64 g2 = mulmod(g, g, m);
  u64 best = g;
  for (u64 k = 1, cur = g; k < two_n / 2; ++k) {
    cur = mulmod(cur, g2, m);  // g^(2k+1)
    if (cur < best) best = cur;
  }
  return best;
}

unsigned bitrev(unsigned x, unsigned bits) { return bits ? __builtin_bitreverse32(x) >> (32 - bits) : 0; }

unsigned bitlen(u64 x) { return x ? 64 - __builtin_clzll(x) : 0; }

}  // namespace he
