"""Seeded synthetic inputs shared by the test-suite, the benchmark and the oracle.

This module draws random numbers and describes workload shapes.  It holds
none of the HE Mul arithmetic: no NTT, no modular products, no key or
ciphertext formation.  Both the HIP library (through its Python binding) and
the CPU oracle receive the same draws from here, so that their outputs can be
compared bit for bit.

The paper's workload is random messages of N/2 complex numbers (Sec. II,
Table I setting); the workload configurations below fix ring size, limb
counts and key-switching digits.
"""
from __future__ import annotations

import dataclasses

import numpy as np

SIGMA = 3.2          # Gaussian error width (Sec. III-A)
TAIL = 6.0           # Gaussian tail cut in units of sigma


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape of one HE Mul workload.

    log_n: ring degree N = 2^log_n; L: q-primes; K: special primes;
    dnum: key-switching digits; q_bits: bit size of each q_i (len L);
    p_bits: bit size of each special prime; h: secret Hamming weight;
    log_scale: log2 of the encoding scale Delta.
    """
    name: str
    log_n: int
    L: int
    K: int
    dnum: int
    q_bits: tuple
    p_bits: int
    h: int
    log_scale: int

    @property
    def N(self) -> int:
        return 1 << self.log_n

    @property
    def alpha(self) -> int:
        return -(-self.L // self.dnum)

    @property
    def slots(self) -> int:
        return self.N // 2


def _mk(name, log_n, L, K, dnum, h, log_scale, first_bits, rest_bits, p_bits):
    return Workload(name, log_n, L, K, dnum, (first_bits,) + (rest_bits,) * (L - 1), p_bits, h, log_scale)


# Plain HE Mul, N=2^12, three ~50-bit q-primes, one ~60-bit special prime.
CFG_N12 = _mk("n12_L3", 12, 3, 1, 3, 64, 40, 50, 50, 60)
# Plain HE Mul, N=2^16, L=24 (q0 60-bit, others 50-bit), dnum=3, K=8 special primes.
CFG_N16 = _mk("n16_L24", 16, 24, 8, 3, 192, 40, 60, 50, 60)
# Plain HE Mul, N=2^17, L=45, dnum=3, K=15.
CFG_N17 = _mk("n17_L45", 17, 45, 15, 3, 192, 50, 60, 50, 60)
# Serving ring N=2^15: L=12, dnum=3, K=4.
CFG_N15 = _mk("n15_L12", 15, 12, 4, 3, 192, 40, 60, 50, 60)
# Tiny rings used by big-integer pins.
CFG_TINY = _mk("n16_tiny", 4, 5, 2, 3, 4, 20, 50, 50, 60)
# The paper's GPU word size (beta = 2^32, primes below 2^30, Table VI) at
# N=2^16: L=40 primes of 30 bits (log Q = 1200, the paper's), dnum=4,
# K=11 special primes of 30 bits, scale 2^30 (one prime per rescale).
CFG_N16_W30 = _mk("n16_L40_w30", 16, 40, 11, 4, 192, 30, 30, 30, 30)
# A small ring of the same prime size for quick parity cases: N=2^12, L=6
# primes of 30 bits, dnum=2 (digits of 3 primes), K=4 special primes.
CFG_N12_W30 = _mk("n12_L6_w30", 12, 6, 4, 2, 64, 25, 30, 30, 30)

# Key-switching variants at N=2^16, L=24 (Sec. III's evaluation key with
# P ~ Q, and one digit per prime): dnum=1 with K=21 special primes of 60
# bits (P > Q), dnum=L=24 with K=2 (P above the largest prime).
CFG_N16_D1 = _mk("n16_L24_d1", 16, 24, 21, 1, 192, 40, 60, 50, 60)
CFG_N16_DL = _mk("n16_L24_d24", 16, 24, 2, 24, 192, 40, 60, 50, 60)
# Small rings of the same variants for the oracle pins.
CFG_N12_D1 = _mk("n12_L6_d1", 12, 6, 6, 1, 64, 40, 60, 50, 60)
CFG_N12_DL = _mk("n12_L6_d6", 12, 6, 2, 6, 64, 40, 60, 50, 60)
# The widest conversion jobs a context allows: dnum = 1 with one digit of 28
# primes (60 + 27 x 50 bits) and K = 24 special primes of 60 bits (1440 bits
# > 1410): 28 sources in the mod-up conversion, 24 in the mod-down one.
CFG_N12_D1W = _mk("n12_L28_d1", 12, 28, 24, 1, 64, 40, 60, 50, 60)
# Ring degrees 2^13 and 2^14 (128-point blocks sub-transforms): small L.
CFG_N13 = _mk("n13_L4", 13, 4, 2, 2, 64, 40, 60, 50, 60)
CFG_N14 = _mk("n14_L6", 14, 6, 3, 2, 64, 40, 60, 50, 60)

WORKLOADS = {w.name: w for w in (CFG_N12, CFG_N16, CFG_N17, CFG_N15, CFG_TINY, CFG_N16_W30, CFG_N12_W30,
                                 CFG_N16_D1, CFG_N16_DL, CFG_N12_D1, CFG_N12_DL, CFG_N12_D1W, CFG_N13, CFG_N14)}

# Seeds of the measured workload.
SEED_KEYS, SEED_MSG_A, SEED_MSG_B, SEED_ENC_A, SEED_ENC_B = 1, 2, 3, 4, 5


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def uniform_limbs(seed: int, moduli, n: int, stream: int = 0) -> np.ndarray:
    """Uniform residues: array [len(moduli)][n] uint64, row i uniform in [0, moduli[i])."""
    g = rng(seed, stream)
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for i, m in enumerate(moduli):
        out[i] = g.integers(0, int(m), size=n, dtype=np.uint64)
    return out


def random_ciphertext(seed: int, moduli, n: int) -> np.ndarray:
    """A ciphertext-shaped array [2][len(moduli)][n] of uniform residues."""
    return np.stack([uniform_limbs(seed, moduli, n, 0), uniform_limbs(seed, moduli, n, 1)])


def ternary_hwt(seed: int, n: int, h: int) -> np.ndarray:
    """Secret: exactly h nonzero coefficients, each +-1 with equal odds."""
    g = rng(seed, 11)
    s = np.zeros(n, dtype=np.int64)
    pos = g.choice(n, size=h, replace=False)
    s[pos] = g.choice(np.array([-1, 1], dtype=np.int64), size=h)
    return s


def zero_one(seed: int, n: int, stream: int = 12) -> np.ndarray:
    """Encryption randomness: 0 with probability 1/2, +-1 with 1/4 each."""
    g = rng(seed, stream)
    u = g.integers(0, 4, size=n)
    return np.where(u == 0, -1, np.where(u == 1, 1, 0)).astype(np.int64)


def gaussian(seed: int, n: int, stream: int, count: int = 1) -> np.ndarray:
    """Rounded Gaussian errors, sigma 3.2, |e| <= 6 sigma: int64 [count][n]."""
    g = rng(seed, stream)
    out = np.empty((count, n), dtype=np.int64)
    for c in range(count):
        x = np.rint(g.normal(0.0, SIGMA, size=n))
        bad = np.abs(x) > TAIL * SIGMA
        while bad.any():
            x[bad] = np.rint(g.normal(0.0, SIGMA, size=int(bad.sum())))
            bad = np.abs(x) > TAIL * SIGMA
        out[c] = x.astype(np.int64)
    return out


def unit_disk(seed: int, n: int) -> np.ndarray:
    """n complex messages uniform in the unit disk (r = sqrt(U), theta = 2 pi U')."""
    g = rng(seed, 21)
    r = np.sqrt(g.random(n))
    th = 2.0 * np.pi * g.random(n)
    return r * np.exp(1j * th)


@dataclasses.dataclass
class KeyDraws:
    s: np.ndarray        # int64 [N] ternary secret
    e_pk: np.ndarray     # int64 [N]
    e_evk: np.ndarray    # int64 [dnum][N]


def key_draws(w: Workload, seed: int = SEED_KEYS) -> KeyDraws:
    return KeyDraws(s=ternary_hwt(seed, w.N, w.h), e_pk=gaussian(seed, w.N, 13)[0],
                    e_evk=gaussian(seed, w.N, 14, w.dnum))


@dataclasses.dataclass
class EncDraws:
    v: np.ndarray        # int64 [N] in {-1, 0, 1}
    e0: np.ndarray       # int64 [N]
    e1: np.ndarray       # int64 [N]


def enc_draws(w: Workload, seed: int) -> EncDraws:
    e = gaussian(seed, w.N, 15, 2)
    return EncDraws(v=zero_one(seed, w.N), e0=e[0], e1=e[1])


def batch_levels(n_pairs: int = 256, lo: int = 4, hi: int = 24, seed: int = 42) -> np.ndarray:
    """Per-pair levels for the batched workload, uniform over lo..hi inclusive."""
    return rng(seed).integers(lo, hi + 1, size=n_pairs)


# ---------------------------------------------------------------- big-integer (non-RNS) workload
# The paper's own HE Mul: N = 2^16, log Q = 1200 (= 40 levels of log p = 30)
# (Sec. II-A, Table III).
BIG_LOG_N, BIG_LOG_Q, BIG_LOG_P = 16, 1200, 30


def big_words(bits: int) -> int:
    """64-bit words holding a `bits`-bit non-negative integer."""
    return -(-bits // 64)


def uniform_bigint(seed: int, bits: int, n: int, stream: int = 0, words: int = 0) -> np.ndarray:
    """n uniform integers in [0, 2^bits) as little-endian words [words][n] uint64
    (words >= big_words(bits); higher words zero)."""
    W = max(words, big_words(bits))
    g = rng(seed, 100 + stream)
    out = np.zeros((W, n), dtype=np.uint64)
    full, rem = divmod(bits, 64)
    for k in range(full):
        out[k] = g.integers(0, 2**64, size=n, dtype=np.uint64)
    if rem:
        out[full] = g.integers(0, 2**rem, size=n, dtype=np.uint64)
    return out


def big_ciphertext(seed: int, logq: int, n: int, words: int = 0) -> np.ndarray:
    """A ciphertext-shaped [2][words][n] array of uniform coefficients below 2^logq."""
    return np.stack([uniform_bigint(seed, logq, n, 0, words), uniform_bigint(seed, logq, n, 1, words)])


def big_evk(seed: int, logQ: int, n: int) -> np.ndarray:
    """An evaluation-key-shaped [2][words][n] array of uniform coefficients below Q^2."""
    return np.stack([uniform_bigint(seed, 2 * logQ, n, 2), uniform_bigint(seed, 2 * logQ, n, 3)])
