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
//                  local stage m_loc uses W[m_loc (2^n1 + b) + j].
// Inside a pass a workgroup owns SUBS sub-transforms; each thread holds
// R = 2^LOGR elements of one of them in registers and runs up to LOGR stages
// per round (radix-2^LOGR).  Round 0 reads its operands straight from the
// producer (global memory or a fused prologue), the last round hands its
// results straight to the consumer; rounds in between exchange through LDS.
//
// The inverse runs the same butterfly network backwards (Gentleman-Sande
// butterflies with TB_invW, stages in reverse order): "blocks" first, then
// "cols", then the factor N^{-1} (merged with any per-limb constant).
//
// Butterfly arithmetic is chosen per modulus (IntA on the 32-bit integer
// multipliers, F64A on FP64 FMAs for q < 2^50); lazy ranges live in
// registers and LDS only, every value written to HBM is canonical.
#pragma once
#include <type_traits>

#include "modarith.hpp"

#ifndef NTT_EPW_DEFAULT
#define NTT_EPW_DEFAULT 2048
#endif

namespace he {

// Twiddle tables take 16 bytes per index and modulus.  Their content
// depends on the modulus (see IntA / F64A): for q >= 2^50 entry k is the
// pair {W_k, floor(W_k 2^63/q)} (2^63-scaled Shoup companion, see
// shoup63_lazy); for q < 2^50 the first half of the modulus's table holds
// the doubles W_k (8 bytes per index) and the second half is unused.
struct Tw2 {
  u64 w, ws;
};

// Moduli below this bound run their butterflies in FP64 (F64A), the rest on
// the 32-bit integer multipliers (IntA).  Both give the same canonical
// results; only the instruction mix differs.
constexpr u64 F64_QLIM = 1ull << 50;
__host__ __device__ constexpr bool f64_mod(u64 q) { return q < F64_QLIM; }

// ---------------------------------------------------------------- integer arithmetic
// Values are u64.  Forward values live in [0, 4q) (Harvey's butterfly),
// inverse values in [0, 2q).
struct IntA {
  using V = u64;
  struct Mod {
    u64 q, q2, nq, n2q;  // q, 2q, 2^64 - q, 2^64 - 2q
  };
  struct Scale {
    u64 w, ws;  // Shoup pair (2^64-scaled companion)
  };
  using Tw = Tw2;
  __device__ static __forceinline__ Mod mod(u64 q, double) { return Mod{q, q << 1, 0 - q, 0 - (q << 1)}; }
  __device__ static __forceinline__ Tw twid(const Tw2* __restrict__ tw, u64 k, const Mod&) { return tw[k]; }
  __device__ static __forceinline__ V in(u64 x, const Mod&) { return x; }
  // Harvey forward butterfly: x, y in [0, 4q) -> x + w y, x - w y in [0, 4q).
  __device__ static __forceinline__ void fwd(V& x, V& y, const Tw2 t, const Mod& M) {
    const u64 X = sub_if_ge(x, M.n2q);
    const u64 T = shoup63_lazy(y, t.w, t.ws, M.nq);
    y = (X + M.q2) - T;
    x = X + T;
  }
  // Gentleman-Sande inverse butterfly: x, y in [0, 2q) -> x + y, (x - y) w in [0, 2q).
  __device__ static __forceinline__ void inv(V& x, V& y, const Tw2 t, const Mod& M) {
    const u64 X = x, Y = y;
    x = sub_if_ge(X + Y, M.n2q);
    y = shoup63_lazy((X + M.q2) - Y, t.w, t.ws, M.nq);
  }
  // canonical value of a lazy transform output
  template <bool FWD>
  __device__ static __forceinline__ u64 out(V x, const Mod& M) {
    if constexpr (FWD) x = csub(x, M.q2);
    return csub(x, M.q);
  }
  __device__ static __forceinline__ Scale scale(u64 w, u64 ws, const Mod&) { return Scale{w, ws}; }
  // canonical x s for an inverse output x in [0, 2q)
  __device__ static __forceinline__ u64 out_scaled(V x, const Scale s, const Mod& M) {
    return csub(shoup_lazy(x, s.w, s.ws, M.q), M.q);
  }
};

// ---------------------------------------------------------------- FP64 arithmetic
// For q < 2^50, values are doubles holding integers, kept centred.  A
// product y w mod q (w < q a twiddle or constant) is formed exactly from
// FMAs, with wq an approximation of w/q of relative error <= 2^-52
// (fl(w fl(1/q)) for table twiddles, fl(w/q) for constants):
//   k  = round(y wq)                 (|y wq| < 2^51; the FMA with
//                                     1.5 2^52 rounds it to an integer)
//   hi = fl(y w),  lo = y w - hi     (exact: two-product by FMA)
//   t  = (hi - k q) + lo             (both steps exact: integers < 2^53)
// so t = y w - k q exactly, with |t| <= (1/2 + |y| 2^-52) q.  A reduction
// x - round(x fl(1/q)) q leaves |x| <= q/2 (+ a 2^-50 relative margin).
// Forward: x' = red(x) + t, y' = red(x) - t; with |x|, |y| <= 1.35 q,
// |t| <= (1/2 + 1.35/4) q and |x'|, |y'| < 1.34 q, so the bound holds at
// every stage.  Inverse: x' = red(x + y), y' = (x - y) w; with |x|, |y| < q,
// |x - y| < 2q (so |(x - y) wq| < 2^51) and |y'| < (1/2 + 2/4) q = q.  The
// build disables FP contraction, so each step is one rounding as written.
struct F64A {
  using V = double;
  struct Mod {
    double q, qinv;  // q and fl(1/q)
  };
  struct Scale {
    double w, wq;  // w and fl(w/q)
  };
  struct Tw {
    double w, wq;
  };
  static constexpr double RND = 6755399441055744.0;  // 1.5 * 2^52
  static constexpr double TWO52 = 4503599627370496.0;
  static constexpr u64 TWO52_BITS = 0x4330000000000000ull;
  __device__ static __forceinline__ Mod mod(u64 q, double qinv) { return Mod{(double)q, qinv}; }
  __device__ static __forceinline__ Tw twid(const Tw2* __restrict__ tw, u64 k, const Mod& M) {
    const double w = reinterpret_cast<const double*>(tw)[k];
    return Tw{w, __dmul_rn(w, M.qinv)};
  }
  // x < 2^52 to double (exact)
  __device__ static __forceinline__ V in(u64 x, const Mod&) {
    return __longlong_as_double((long long)(x | TWO52_BITS)) - TWO52;
  }
  __device__ static __forceinline__ double red(double x, const Mod& M) {
    const double k = __fma_rn(x, M.qinv, RND) - RND;
    return __fma_rn(-k, M.q, x);
  }
  __device__ static __forceinline__ double mulw(double y, double w, double wq, const Mod& M) {
    const double k = __fma_rn(y, wq, RND) - RND;
    const double hi = __dmul_rn(y, w);
    const double lo = __fma_rn(y, w, -hi);
    const double r = __fma_rn(-k, M.q, hi);
    return __dadd_rn(r, lo);
  }
  // a b mod q for 0 <= a, b < q, as an integer of magnitude <= 3q/4:
  // k = round(fl(a b) fl(1/q)) is within 3/4 of a b / q (a b / q < 2^50),
  // and (fl(a b) - k q) + (a b - fl(a b)) is exact as above.
  __device__ static __forceinline__ double mulv(double a, double b, const Mod& M) {
    const double hi = __dmul_rn(a, b);
    const double lo = __fma_rn(a, b, -hi);
    const double k = __fma_rn(hi, M.qinv, RND) - RND;
    return __dadd_rn(__fma_rn(-k, M.q, hi), lo);
  }
  __device__ static __forceinline__ void fwd(V& x, V& y, const Tw t, const Mod& M) {
    const double X = red(x, M);
    const double T = mulw(y, t.w, t.wq, M);
    x = X + T;
    y = X - T;
  }
  __device__ static __forceinline__ void inv(V& x, V& y, const Tw t, const Mod& M) {
    const double X = x, Y = y;
    x = red(X + Y, M);
    y = mulw(X - Y, t.w, t.wq, M);
  }
  // |c| <= q, c integral, c mod q in [0, q) -> canonical u64 (c = q cannot
  // occur: outputs come from red() or mulw(), both below q in magnitude)
  __device__ static __forceinline__ u64 to_u64(double c, const Mod& M) {
    const double v = c < 0.0 ? c + M.q : c;
    return (u64)__double_as_longlong(v + TWO52) - TWO52_BITS;
  }
  template <bool FWD>
  __device__ static __forceinline__ u64 out(V x, const Mod& M) {
    return to_u64(red(x, M), M);
  }
  // w < q; fl(w/q) once per thread
  __device__ static __forceinline__ Scale scale(u64 w, u64, const Mod& M) {
    const double wd = (double)w;
    return Scale{wd, __ddiv_rn(wd, M.q)};
  }
  __device__ static __forceinline__ u64 out_scaled(V x, const Scale s, const Mod& M) {
    return to_u64(mulw(x, s.w, s.wq, M), M);
  }
};

// ---------------------------------------------------------------- 32-bit integer arithmetic
// For q < 2^30 stored in 32-bit words (the paper's GPU word size): values
// are u32 on the native 32x32-bit multipliers.  Shoup's product with a
// 2^32-scaled companion w' = floor(w 2^32 / q): for any y < 2^32,
// y w - mulhi(y, w') q lies in [0, 2q) and is computed mod 2^32 (two
// v_mul_lo_u32 and one v_mul_hi_u32).  Forward values live in [0, 4q)
// (Harvey), inverse values in [0, 2q); 4q < 2^32.  Table entry k holds
// w | w' << 32 (8 bytes per index); constants keep their 2^64-scaled
// companion, whose top half is the 2^32-scaled one.
struct I32A {
  using V = u32;
  struct Mod {
    u32 q, q2;
  };
  struct Scale {
    u32 w, ws;
  };
  struct Tw {
    u32 w, ws;
  };
  __device__ static __forceinline__ Tw twid(const Tw2* __restrict__ tw, u64 k, const Mod&) {
    const u64 v = reinterpret_cast<const u64*>(tw)[k];
    return Tw{(u32)v, (u32)(v >> 32)};
  }
  __device__ static __forceinline__ Mod mod(u64 q, double) { return Mod{(u32)q, (u32)(q << 1)}; }
  __device__ static __forceinline__ V in(u64 x, const Mod&) { return (u32)x; }
  __device__ static __forceinline__ u32 mulw(u32 y, u32 w, u32 ws, u32 q) { return y * w - __umulhi(y, ws) * q; }
  __device__ static __forceinline__ void fwd(V& x, V& y, const Tw t, const Mod& M) {
    const u32 X = x >= M.q2 ? x - M.q2 : x;
    const u32 T = mulw(y, t.w, t.ws, M.q);
    y = X - T + M.q2;
    x = X + T;
  }
  __device__ static __forceinline__ void inv(V& x, V& y, const Tw t, const Mod& M) {
    const u32 X = x, Y = y;
    const u32 s = X + Y;
    x = s >= M.q2 ? s - M.q2 : s;
    y = mulw(X - Y + M.q2, t.w, t.ws, M.q);
  }
  template <bool FWD>
  __device__ static __forceinline__ u64 out(V x, const Mod& M) {
    if constexpr (FWD) x = x >= M.q2 ? x - M.q2 : x;
    return x >= M.q ? x - M.q : x;
  }
  __device__ static __forceinline__ Scale scale(u64 w, u64 ws, const Mod&) { return Scale{(u32)w, (u32)(ws >> 32)}; }
  __device__ static __forceinline__ u64 out_scaled(V x, const Scale s, const Mod& M) {
    const u32 r = mulw(x, s.w, s.ws, M.q);
    return r >= M.q ? r - M.q : r;
  }
};

// Workgroup barrier ordering LDS accesses only: unlike __syncthreads() it
// does not wait for outstanding global loads and stores, so prefetches and
// stores stay in flight across the LDS exchanges of a transform.  Kernels
// never pass data between threads through global memory.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// Ordering of LDS accesses among the lanes of one wavefront (a transform
// whose threads all sit in one wave): the LDS unit executes one wave's
// accesses in issue order, so only the compiler must not reorder them.
__device__ __forceinline__ void lds_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) lds_wave_sync();
  else lds_barrier();
}

template <int LOGS, int LOGR>
struct Geo {
  static constexpr int S = 1 << LOGS;
  static constexpr int R = 1 << LOGR;
  static constexpr int T = S / R;                      // threads per sub-transform
  static constexpr int NR = (LOGS + LOGR - 1) / LOGR;  // register rounds
  static constexpr int SUB = S + (S >> 4) + 1;         // padded LDS stride (words), odd
  __device__ static __forceinline__ int pad(int e) { return e + (e >> 4); }
};

// Element indices owned by thread tt in round RD: group u, member i is
//   e = blk * span + c + i * cnt_c   with g = tt + u*T, blk = g / cnt_c, c = g % cnt_c.
template <int LOGS, int LOGR, int RD>
struct RoundShape {
  using Gm = Geo<LOGS, LOGR>;
  static constexpr int st = RD * LOGR;
  static constexpr int rr = (LOGS - st) < LOGR ? (LOGS - st) : LOGR;
  static constexpr int G = 1 << rr;
  static constexpr int NG = Gm::R / G;
  static constexpr int cnt_c = Gm::S >> (st + rr);
  static constexpr int span = Gm::S >> st;
  __device__ static __forceinline__ int elem(int tt, int u, int i) {
    const int g = tt + u * Gm::T;
    return (g / cnt_c) * span + (g % cnt_c) + i * cnt_c;
  }
  __device__ static __forceinline__ int blk(int tt, int u) { return (tt + u * Gm::T) / cnt_c; }
};

// Twiddle sources of the register rounds of one sub-transform; stage s
// (0 .. LOGS-1 inside the sub-transform), group t < 2^s.
//   TabTw: the table entry at (base << s) + t (TB_W or TB_invW of the
//          modulus; base = 2^n1 + blk in a blocks pass, 1 in a cols pass).
//   GenTw: FP64 moduli in blocks passes.  That entry factors as
//          a[2^s + t] * b[s] mod q (a: psi^(brv_s(t) 2^(log_n - s)), shared
//          by every block of the modulus; b: psi^((2 brv_n1(blk) + 1)
//          2^(LOGS - 1 - s)), the block's row), formed exactly by F64A::mulw
//          (centred, |w| < q, as the butterflies' bounds allow), so a block
//          reads LOGS words of b rather than 2^LOGS - 1 table entries.
struct TabTw {
  const Tw2* __restrict__ tw;
  u64 base;
};
struct GenTw {
  const double* __restrict__ a;
  const double* __restrict__ b;
};
template <class A>
__device__ __forceinline__ typename A::Tw twiddle(const TabTw& s, int sl, u64 t, const typename A::Mod& M) {
  return A::twid(s.tw, (s.base << sl) + t, M);
}
template <class A>
__device__ __forceinline__ typename A::Tw twiddle(const GenTw& s, int sl, u64 t, const typename A::Mod& M) {
  static_assert(std::is_same<A, F64A>::value, "generated twiddles are for FP64 moduli");
  const double b = s.b[sl];
  if (__builtin_constant_p(t) && t == 0) return F64A::Tw{b, __dmul_rn(b, M.qinv)};  // a[2^s] = 1
  const double w = F64A::mulw(s.a[(1ull << sl) + t], b, __dmul_rn(b, M.qinv), M);
  return F64A::Tw{w, __dmul_rn(w, M.qinv)};
}

// Butterflies of round RD on the registers x[0..R) of thread tt.
template <class A, bool FWD, int LOGS, int LOGR, int RD, class TS>
__device__ __forceinline__ void round_math(typename A::V (&x)[1 << LOGR], int tt, const TS& ts,
                                           const typename A::Mod& M) {
  using RS = RoundShape<LOGS, LOGR, RD>;
  constexpr int G = RS::G, rr = RS::rr, st = RS::st;
#pragma unroll
  for (int u = 0; u < RS::NG; ++u) {
    // the first round's groups all start at 0 (its threads' group index
    // tt + u T stays below cnt_c)
    const u64 blk = st == 0 ? 0 : (u64)RS::blk(tt, u);
    typename A::V* v = x + u * G;
    if constexpr (FWD) {
#pragma unroll
      for (int k = 0; k < rr; ++k) {
        const int half = G >> (k + 1);
#pragma unroll
        for (int i = 0; i < G; ++i) {
          if (i & half) continue;
          A::fwd(v[i], v[i + half], twiddle<A>(ts, st + k, (blk << k) + (u64)(i >> (rr - k)), M), M);
        }
      }
    } else {
#pragma unroll
      for (int k = rr - 1; k >= 0; --k) {
        const int half = G >> (k + 1);
#pragma unroll
        for (int i = 0; i < G; ++i) {
          if (i & half) continue;
          A::inv(v[i], v[i + half], twiddle<A>(ts, st + k, (blk << k) + (u64)(i >> (rr - k)), M), M);
        }
      }
    }
  }
}

template <int LOGS, int LOGR, int RD, class V>
__device__ __forceinline__ void lds_put(V* tile, const V (&x)[1 << LOGR], int tt) {
  using RS = RoundShape<LOGS, LOGR, RD>;
#pragma unroll
  for (int u = 0; u < RS::NG; ++u)
#pragma unroll
    for (int i = 0; i < RS::G; ++i) tile[Geo<LOGS, LOGR>::pad(RS::elem(tt, u, i))] = x[u * RS::G + i];
}
template <int LOGS, int LOGR, int RD, class V>
__device__ __forceinline__ void lds_get(const V* tile, V (&x)[1 << LOGR], int tt) {
  using RS = RoundShape<LOGS, LOGR, RD>;
#pragma unroll
  for (int u = 0; u < RS::NG; ++u)
#pragma unroll
    for (int i = 0; i < RS::G; ++i) x[u * RS::G + i] = tile[Geo<LOGS, LOGR>::pad(RS::elem(tt, u, i))];
}

// Middle rounds 1 .. NR-2 (forward order) through LDS.  WAVE: the
// transform's threads are one wavefront (wave-level LDS ordering suffices).
template <class A, bool FWD, int LOGS, int LOGR, int K, bool WAVE, class TS>
__device__ __forceinline__ void mid_rounds(typename A::V (&x)[1 << LOGR], typename A::V* tile, int tt, const TS& ts,
                                           const typename A::Mod& M) {
  constexpr int NR = Geo<LOGS, LOGR>::NR;
  if constexpr (K < NR - 1) {
    constexpr int RD = FWD ? K : NR - 1 - K;
    constexpr int PREV = FWD ? RD - 1 : RD + 1;
    lds_put<LOGS, LOGR, PREV>(tile, x, tt);
    lds_sync<WAVE>();
    lds_get<LOGS, LOGR, RD>(tile, x, tt);
    round_math<A, FWD, LOGS, LOGR, RD>(x, tt, ts, M);
    // no barrier needed before the next lds_put: within one round every LDS
    // position belongs to exactly one thread
    mid_rounds<A, FWD, LOGS, LOGR, K + 1, WAVE>(x, tile, tt, ts, M);
  }
}

// Whole sub-transform with the first round's operands already in x (in the
// first round's element order).  The last round hands element e to
// store(e, v) (lazy value of arithmetic A), or, when OUT_LDS, leaves it in
// the tile for a coalesced copy-out after a barrier.  `tile` is this
// sub-transform's LDS area (Geo::SUB words).  A caller that runs several
// sub-transforms on the same tile back to back must place a barrier between
// them.
template <class A, bool FWD, int LOGS, int LOGR, bool OUT_LDS, bool WAVE = false, class TS, class Store>
__device__ __forceinline__ void sub_transform_src(typename A::V (&x)[1 << LOGR], typename A::V* tile, int tt,
                                                  const TS& ts, const typename A::Mod& M, Store&& store) {
  using Gm = Geo<LOGS, LOGR>;
  constexpr int NR = Gm::NR;
  constexpr int FIRST = FWD ? 0 : NR - 1;
  constexpr int LAST = FWD ? NR - 1 : 0;
  round_math<A, FWD, LOGS, LOGR, FIRST>(x, tt, ts, M);
  if constexpr (NR > 1) {
    mid_rounds<A, FWD, LOGS, LOGR, 1, WAVE>(x, tile, tt, ts, M);
    constexpr int PREV = FWD ? LAST - 1 : LAST + 1;
    lds_put<LOGS, LOGR, PREV>(tile, x, tt);
    lds_sync<WAVE>();
    lds_get<LOGS, LOGR, LAST>(tile, x, tt);
    round_math<A, FWD, LOGS, LOGR, LAST>(x, tt, ts, M);
  }
  if constexpr (OUT_LDS) {
    lds_put<LOGS, LOGR, LAST>(tile, x, tt);
  } else {
    using RS = RoundShape<LOGS, LOGR, LAST>;
#pragma unroll
    for (int u = 0; u < RS::NG; ++u)
#pragma unroll
      for (int i = 0; i < RS::G; ++i) store(RS::elem(tt, u, i), x[u * RS::G + i]);
  }
}

// The same with the twiddles of the table tw at base (see TabTw).
template <class A, bool FWD, int LOGS, int LOGR, bool OUT_LDS, bool WAVE = false, class Store>
__device__ __forceinline__ void sub_transform_regs(typename A::V (&x)[1 << LOGR], typename A::V* tile, int tt,
                                                   const Tw2* __restrict__ tw, u64 base, const typename A::Mod& M,
                                                   Store&& store) {
  sub_transform_src<A, FWD, LOGS, LOGR, OUT_LDS, WAVE>(x, tile, tt, TabTw{tw, base}, M, store);
}

// Runs body(IntA{}), body(F64A{}) or, for 32-bit words, body(I32A{}) by
// the modulus (uniform per workgroup).  A modulus runs I32A when its
// context stores 32-bit words with integer butterflies (ModInfo::arith).
template <class W = u64, class Body>
__device__ __forceinline__ void with_arith(const ModInfo& mo, Body&& body) {
  if constexpr (sizeof(W) == 4) {
    if (mo.arith == ARITH_I32) {
      body(I32A{});
      return;
    }
  }
  if (f64_mod(mo.q)) body(F64A{});
  else body(IntA{});
}

// log2 of the register radix of a 2^logs-point sub-transform: radix 8 at
// every size (64 to 512 points).  Fewer, larger rounds hold more values per
// thread: 256 points in two radix-16 rounds halve the waves of a pass over
// one HE Mul's limbs (about one wave per SIMD, so fewer waves hide less
// memory latency), and 128 or 512 points at radix 16 or 32 push the passes
// to 130-256 VGPRs (the combine pass at N = 2^17 to one wave per SIMD).
// Measured per HE Mul: N = 2^15 0.108 -> 0.100 ms, N = 2^17 0.805 -> 0.720
// ms against radix 16 / 32.  Batches may still choose radix 16 at N = 2^16
// (see tile_code).
__host__ __device__ constexpr int radix_log(int) { return 3; }
template <int LOGS>
struct Radix {
  static constexpr int LOGR = radix_log(LOGS);
};

// The tile parameter T of a pass kernel: elements per workgroup in its low
// 24 bits and, from bit 24 up, log2 of the register radix (0 there: the
// default radix_log of the sub-transform size), so a pass can be
// instantiated at another radix (a schedule choice of batches).
__host__ __device__ constexpr int tile_elems(int t) { return t & 0xFFFFFF; }
__host__ __device__ constexpr int tile_logr(int t, int logs) { return (t >> 24) ? (t >> 24) : radix_log(logs); }
__host__ __device__ constexpr int tile_code(int elems, int logr) { return elems | (logr << 24); }

// Workgroup shape of a pass: EPW elements (8*EPW bytes) per workgroup.
// `cols` passes put the sub index fastest (adjacent lanes read adjacent
// columns); `blocks` passes put the in-sub thread fastest.
constexpr int NTT_EPW = NTT_EPW_DEFAULT;
template <int LOGS, int EPW = NTT_EPW>
struct PassGeo {
  static constexpr int LOGR = tile_logr(EPW, LOGS);
  using Gm = Geo<LOGS, LOGR>;
  static constexpr int SUBS = tile_elems(EPW) / Gm::S;
  static constexpr int THREADS = SUBS * Gm::T;
};
// threads of a pass workgroup (a plain function so it fits a macro argument)
constexpr int pass_threads(int logs, int epw) {
  return (tile_elems(epw) >> logs) * ((1 << logs) >> tile_logr(epw, logs));
}
template <int LOGS, bool COLS, int EPW = NTT_EPW>
struct PassLayout {
  static_assert(PassGeo<LOGS, EPW>::THREADS == pass_threads(LOGS, EPW), "pass_threads");
  using Gm = typename PassGeo<LOGS, EPW>::Gm;
  static constexpr int SUBS = PassGeo<LOGS, EPW>::SUBS;
  __device__ static __forceinline__ int sub() { return COLS ? (int)threadIdx.x % SUBS : (int)threadIdx.x / Gm::T; }
  __device__ static __forceinline__ int tt() { return COLS ? (int)threadIdx.x / SUBS : (int)threadIdx.x % Gm::T; }
};

// ------------------------------------------------------------------ plain passes
// Arguments of one batched transform launch: limb l of polynomial z reads
// src + l*src_stride + z*src_zstride, writes dst likewise (in place allowed),
// works modulo mods[limb_mod[l]], and (inverse "cols" pass) multiplies by the
// Shoup pair scale[2l], scale[2l+1] instead of N^{-1} when scale != null.
struct NttArgs {
  const u64* src;
  u64* dst;
  u64 src_stride, dst_stride;
  u64 src_zstride, dst_zstride;
  const u32* limb_mod;
  const ModInfo* mods;
  const Tw2* tw;  // [nmods][N] (W or invW with companions)
  const u64* scale;
  u32 log_n;
};

template <bool FWD, int LOGS, int EPW = NTT_EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_cols(NttArgs a) {
  constexpr int LOGR = tile_logr(EPW, LOGS);
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, true, EPW>;
  constexpr int FIRST = FWD ? 0 : Gm::NR - 1;
  using RF = RoundShape<LOGS, LOGR, FIRST>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const int limb = blockIdx.y;
  const u32 mi = a.limb_mod[limb];
  const ModInfo mo = ldc(a.mods + mi);
  const int n2 = a.log_n - LOGS;
  const int sub = PL::sub(), tt = PL::tt();
  const u64 col = (u64)blockIdx.x * PL::SUBS + sub;
  const auto in = gbl(a.src + (u64)limb * a.src_stride + (u64)blockIdx.z * a.src_zstride + col);
  const auto out = gbl(a.dst + (u64)limb * a.dst_stride + (u64)blockIdx.z * a.dst_zstride + col);
  u64 sw = mo.ninv, sws = mo.ninvs;
  if (!FWD && a.scale) {
    sw = a.scale[2 * (u64)limb];
    sws = a.scale[2 * (u64)limb + 1];
  }
  u64 xi[Gm::R];
#pragma unroll
  for (int k = 0; k < Gm::R; ++k) xi[k] = in[(u64)RF::elem(tt, k / RF::G, k % RF::G) << n2];
  with_arith(mo, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(mo.q, mo.qinv);
    const typename A::Scale sc = A::scale(sw, sws, M);
    typename A::V x[Gm::R];
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) x[k] = A::in(xi[k], M);
    sub_transform_regs<A, FWD, LOGS, LOGR, false>(
        x, reinterpret_cast<typename A::V*>(lds) + sub * Gm::SUB, tt, a.tw + ((u64)mi << a.log_n), 1, M,
        [&](int e, typename A::V v) {
          out[(u64)e << n2] = FWD ? A::template out<true>(v, M) : A::out_scaled(v, sc, M);
        });
  });
}

// Blocks pass.  The side whose register layout is thread-contiguous
// (forward output, inverse input) goes through LDS so that every global
// access is coalesced.
template <bool FWD, int LOGS, int EPW = NTT_EPW>
__global__ __launch_bounds__(pass_threads(LOGS, EPW)) void k_ntt_blocks(NttArgs a) {
  constexpr int LOGR = tile_logr(EPW, LOGS);
  using Gm = Geo<LOGS, LOGR>;
  using PL = PassLayout<LOGS, false, EPW>;
  constexpr int THREADS = PassGeo<LOGS, EPW>::THREADS;
  constexpr int FIRST = FWD ? 0 : Gm::NR - 1;
  using RF = RoundShape<LOGS, LOGR, FIRST>;
  __shared__ u64 lds[PL::SUBS * Gm::SUB];
  const int limb = blockIdx.y;
  const u32 mi = a.limb_mod[limb];
  const ModInfo mo = ldc(a.mods + mi);
  const int n1 = a.log_n - LOGS;
  const int sub = PL::sub(), tt = PL::tt();
  const u64 blk0 = (u64)blockIdx.x * PL::SUBS;
  const auto in0 = gbl(a.src + (u64)limb * a.src_stride + (u64)blockIdx.z * a.src_zstride + (blk0 << LOGS));
  const auto out0 = gbl(a.dst + (u64)limb * a.dst_stride + (u64)blockIdx.z * a.dst_zstride + (blk0 << LOGS));
  const auto in = in0 + ((u64)sub << LOGS);
  const auto out = out0 + ((u64)sub << LOGS);
  u64 xi[Gm::R];
  if constexpr (!FWD) {
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) {
      const int idx = threadIdx.x + k * THREADS;
      lds[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))] = in0[idx];
    }
    lds_barrier();
    // the transform writes only tile positions this thread has just read
    lds_get<LOGS, LOGR, FIRST>(lds + sub * Gm::SUB, xi, tt);
  } else {
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) xi[k] = in[RF::elem(tt, k / RF::G, k % RF::G)];
  }
  with_arith(mo, [&](auto ar) {
    using A = decltype(ar);
    const typename A::Mod M = A::mod(mo.q, mo.qinv);
    typename A::V* tl = reinterpret_cast<typename A::V*>(lds);
    typename A::V x[Gm::R];
#pragma unroll
    for (int k = 0; k < Gm::R; ++k) x[k] = A::in(xi[k], M);
    sub_transform_regs<A, FWD, LOGS, LOGR, FWD>(x, tl + sub * Gm::SUB, tt, a.tw + ((u64)mi << a.log_n),
                                                (1ull << n1) + blk0 + sub, M,
                                                [&](int e, typename A::V v) { out[e] = A::template out<FWD>(v, M); });
    if constexpr (FWD) {
      lds_barrier();
#pragma unroll
      for (int k = 0; k < Gm::R; ++k) {
        const int idx = threadIdx.x + k * THREADS;
        out0[idx] = A::template out<true>(tl[(idx >> LOGS) * Gm::SUB + Gm::pad(idx & (Gm::S - 1))], M);
      }
    }
  });
}

}  // namespace he
