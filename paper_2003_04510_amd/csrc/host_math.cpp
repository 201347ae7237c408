#include "host_math.hpp"

namespace he {

u64 powmod(u64 a, u64 e, u64 m) {
  u64 r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
    e >>= 1;
  }
  return r;
}

// Miller-Rabin with the first twelve primes as bases: exact below 3.3e24.
bool is_prime(u64 n) {
  const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (u64 b : bases)
    if (n % b == 0) return n == b;
  u64 d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  for (u64 b : bases) {
    u64 x = powmod(b, d, n);
    if (x == 1 || x == n - 1) continue;
    bool witness = true;
    for (int r = 1; r < s && witness; ++r) {
      x = mulmod(x, x, n);
      if (x == n - 1) witness = false;
    }
    if (witness) return false;
  }
  return true;
}

bool gen_primes(unsigned log_n, unsigned bits, unsigned count, const u64* excl, unsigned nexcl,
                u64* out) {
  const u64 step = 2ull << log_n;
  const u64 top = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
  u64 x = top / step * step + 1;
  if (x > top) x -= step;
  unsigned found = 0;
  while (found < count && x > step) {
    if (is_prime(x)) {
      bool skip = false;
      for (unsigned i = 0; i < nexcl; ++i) skip |= (excl[i] == x);
      if (!skip) out[found++] = x;
    }
    x -= step;
  }
  return found == count;
}

u64 min_root_2n(u64 m, unsigned log_n) {
  const u64 n = 1ull << log_n, two_n = 2 * n;
  if ((m - 1) % two_n) return 0;
  u64 g = 0;
  for (u64 c = 2; c < m && !g; ++c) {
    u64 r = powmod(c, (m - 1) / two_n, m);
    if (powmod(r, n, m) == m - 1) g = r;  // order exactly 2N
  }
  // primitive 2N-th roots are the odd powers of g; take the least
  u64 best = g, cur = g;
  const u64 g2 = mulmod(g, g, m);
  for (u64 k = 3; k < two_n; k += 2) {
    cur = mulmod(cur, g2, m);
    if (cur < best) best = cur;
  }
  return best;
}

unsigned bitrev(unsigned x, unsigned bits) {
  unsigned r = 0;
  for (unsigned i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

unsigned bitlen(u64 x) {
  unsigned b = 0;
  while (x) { ++b; x >>= 1; }
  return b;
}

}  // namespace he
