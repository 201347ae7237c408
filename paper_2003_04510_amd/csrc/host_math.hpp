// Host-side number theory for the RNS bases: primality, prime search,
// primitive roots, modular inverses, Shoup/Barrett companions.
#pragma once
#include <cstdint>
#include <vector>

namespace he {

using u64 = uint64_t;
using u128 = unsigned __int128;

inline u64 mulmod(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }
inline u64 addmod(u64 a, u64 b, u64 m) { u64 s = a + b; return s >= m ? s - m : s; }
inline u64 submod(u64 a, u64 b, u64 m) { return a >= b ? a - b : a + m - b; }
u64 powmod(u64 a, u64 e, u64 m);
inline u64 invmod(u64 a, u64 m) { return powmod(a % m, m - 2, m); }  // m prime
// Shoup companion floor(w * 2^64 / m), w < m  (the paper's Y_Shoup, Algorithm 2)
inline u64 shoup(u64 w, u64 m) { return (u64)(((u128)w << 64) / m); }
// 2^63-scaled companion floor(w * 2^63 / m) used by the NTT butterflies
inline u64 shoup63(u64 w, u64 m) { return (u64)(((u128)w << 63) / m); }
bool is_prime(u64 n);
// The `count` largest primes below 2^bits that are 1 mod 2N, scanning down.
bool gen_primes(unsigned log_n, unsigned bits, unsigned count, const u64* excl, unsigned nexcl,
                u64* out);
// Smallest primitive 2N-th root of unity mod prime m (m = 1 mod 2N).
u64 min_root_2n(u64 m, unsigned log_n);
unsigned bitrev(unsigned x, unsigned bits);
unsigned bitlen(u64 x);

}  // namespace he
