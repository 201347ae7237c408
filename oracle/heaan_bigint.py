"""CPU oracle for the paper's non-RNS HEAAN HE Mul -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The HIP library never imports it and shares no code
with it.

The paper (Sec. II and III, Fig. 2) describes HEAAN with power-of-two moduli:
a ciphertext (bx, ax) at level q = 2^logq holds two polynomials of
Z[X]/(X^N + 1) whose coefficients are big integers in [0, q); the
evaluation key holds two polynomials modulo Q^2 (Q = 2^logQ) that encrypt
Q * sk^2.  HE Mul multiplies and adds the input polynomials (region 1) and
key-switches the ax*ax term with the evaluation key (region 2), whose
products are shifted right by log Q; rescaling divides by p = 2^logp.

Everything here is exact integer arithmetic on Python ints:
  * the negacyclic product over Z by Kronecker substitution (each polynomial
    packed into one integer with a slot wide enough that no slot overflows;
    Python's integer product is the library step), then X^N = -1 folding;
  * reductions mod 2^k as masks (Python's & on negative ints keeps the
    two's-complement residue, i.e. the value mod 2^k);
  * shifts with rounding as floor((x + 2^(k-1)) / 2^k) of the non-negative
    residue.

Readings (the paper is silent on them; HEAAN's published description is
followed): region 1 uses three products (ax1+bx1)(ax2+bx2), ax1 ax2, bx1 bx2
(five polynomial products in all, with the two of region 2); the key-switch
shift and the rescale round half up; the paper's sign convention
c.bx = c.ax * sk + t + e fixes decryption as t = bx - ax * sk and the key as
evk.bx = evk.ax * sk + e + Q sk^2 (mod Q^2).

Pins: tests/test_oracle_bigint_pins.py (schoolbook products over Z, X^j
shifts, the Karatsuba identity, exact rounding of the shifts, the
decryption identity decrypt(c1 * c2) ~ decrypt(c1) * decrypt(c2) within the
key-switching error bound, and he_mul_at -- coefficient by coefficient from
direct sums -- against he_mul's Kronecker products at small N).
"""
from __future__ import annotations

import numpy as np


def mask(bits: int) -> int:
    return (1 << bits) - 1


def _pack(a, slot: int) -> int:
    """sum_i a_i 2^(slot i) for non-negative a_i < 2^slot (slot a multiple of 8)."""
    nb = slot // 8
    return int.from_bytes(b"".join(int(x).to_bytes(nb, "little") for x in a), "little")


def _unpack(x: int, slot: int, count: int) -> list:
    nb = slot // 8
    raw = x.to_bytes(nb * count, "little")
    return [int.from_bytes(raw[i * nb:(i + 1) * nb], "little") for i in range(count)]


def negacyclic_mul(a, b) -> list:
    """Exact c = a * b in Z[X]/(X^N + 1) for non-negative integer coefficients.

    c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j  (Sec. II: polynomial
    mul in the cyclotomic ring).  The full product of degree 2N-2 comes from
    one integer product of the packed operands."""
    n = len(a)
    assert len(b) == n and n >= 1
    assert min(a) >= 0 and min(b) >= 0
    ba = max(int(x).bit_length() for x in a)
    bb = max(int(x).bit_length() for x in b)
    slot = ba + bb + n.bit_length() + 1
    slot = -(-slot // 64) * 64
    full = _unpack(_pack(a, slot) * _pack(b, slot), slot, 2 * n)
    return [full[k] - full[k + n] for k in range(n)]


def he_mul(ct1, ct2, evk, logq: int, logQ: int):
    """HEAAN HE Mul at level q = 2^logq (Fig. 2): returns (bx3, ax3).

    ct = (bx, ax), lists of ints in [0, 2^logq); evk = (evk.bx, evk.ax),
    lists of ints in [0, 2^(2 logQ)).
      region 1: axbx = (ax1+bx1)(ax2+bx2), axax = ax1 ax2, bxbx = bx1 bx2 mod q
      region 2: ks_u = round((axax * evk_u mod qQ) / Q) mod q, u in {bx, ax}
      ax3 = ks_ax + axbx - axax - bxbx, bx3 = ks_bx + bxbx (mod q)."""
    assert logq <= logQ
    qm = mask(logq)
    bx1, ax1 = ct1
    bx2, ax2 = ct2
    s1 = [(x + y) & qm for x, y in zip(ax1, bx1)]
    s2 = [(x + y) & qm for x, y in zip(ax2, bx2)]
    axbx = [c & qm for c in negacyclic_mul(s1, s2)]
    axax = [c & qm for c in negacyclic_mul(ax1, ax2)]
    bxbx = [c & qm for c in negacyclic_mul(bx1, bx2)]
    ks = [key_switch_part(axax, e, logq, logQ) for e in evk]
    ax3 = [(k + p - x - y) & qm for k, p, x, y in zip(ks[1], axbx, axax, bxbx)]
    bx3 = [(k + y) & qm for k, y in zip(ks[0], bxbx)]
    return bx3, ax3


def key_switch_part(axax, evk_u, logq: int, logQ: int) -> list:
    """round((axax * evk_u mod 2^(logq+logQ)) / 2^logQ) mod 2^logq (region 2's shift)."""
    qq = mask(logq + logQ)
    half = 1 << (logQ - 1)
    return [(((c & qq) + half) >> logQ) & mask(logq) for c in negacyclic_mul(axax, evk_u)]


def rescale(ct, logq: int, logp: int):
    """Divide by p = 2^logp with rounding: level q -> q / p (Sec. II-A)."""
    half = 1 << (logp - 1)
    m = mask(logq - logp)
    return tuple([((c + half) >> logp) & m for c in poly] for poly in ct)


# ---------------------------------------------------------------- chosen output coefficients
def negacyclic_coeff(a, b_terms, k: int, n: int) -> int:
    """Coefficient k of a * b in Z[X]/(X^N + 1), N = n, with b given as its
    nonzero terms {j: b_j}: sum_j a_{k-j} b_j for j <= k, and -a_{k-j+N} b_j
    for j > k (X^N = -1).  O(number of terms)."""
    c = 0
    for j, bj in b_terms.items():
        if j <= k:
            c += a[k - j] * bj
        else:
            c -= a[k - j + n] * bj
    return c


def _terms(a) -> dict:
    return {j: int(x) for j, x in enumerate(a) if x}


def he_mul_at(ct1, ct2, evk, logq: int, logQ: int, idx, logp: int = 0):
    """Coefficients idx of HE Mul (as he_mul, then rescale by 2^logp when
    logp > 0), each computed on its own from the definitions of region 1
    and region 2 by direct negacyclic sums: the products with ct2's
    polynomials cost their nonzero terms per coefficient (cheap when ct2 is
    sparse); the key switch needs every coefficient of ax1 ax2 and one sum
    of N products per output coefficient.  Returns (bx3, ax3) at idx."""
    n = len(ct1[0])
    qm = mask(logq)
    bx1, ax1 = ct1
    bx2, ax2 = ct2
    s1 = [(int(x) + int(y)) & qm for x, y in zip(ax1, bx1)]
    t_s2 = _terms([(int(x) + int(y)) & qm for x, y in zip(ax2, bx2)])
    t_ax2, t_bx2 = _terms(ax2), _terms(bx2)
    ax1i = [int(x) for x in ax1]
    bx1i = [int(x) for x in bx1]
    axax = [negacyclic_coeff(ax1i, t_ax2, k, n) & qm for k in range(n)]
    qq, half = mask(logq + logQ), 1 << (logQ - 1)
    ev = [[int(x) for x in e] for e in evk]
    bx3, ax3 = [], []
    for k in idx:
        axbx = negacyclic_coeff(s1, t_s2, k, n) & qm
        bxbx = negacyclic_coeff(bx1i, t_bx2, k, n) & qm
        ks = []
        for e in ev:
            c = sum(axax[i] * e[k - i] for i in range(k + 1)) - sum(axax[i] * e[k - i + n] for i in range(k + 1, n))
            ks.append((((c & qq) + half) >> logQ) & qm)
        bx3.append((ks[0] + bxbx) & qm)
        ax3.append((ks[1] + axbx - axax[k] - bxbx) & qm)
    if logp > 0:
        hp, mo = 1 << (logp - 1), mask(logq - logp)
        bx3 = [((c + hp) >> logp) & mo for c in bx3]
        ax3 = [((c + hp) >> logp) & mo for c in ax3]
    return bx3, ax3


# ---------------------------------------------------------------- keys and encryption
def evk_from_secret(s, a, e, logQ: int):
    """evk = (evk.bx, evk.ax) with evk.bx = a s + e + Q s^2 (mod Q^2), evk.ax = a.

    s, e: small signed integer polynomials; a: ints in [0, Q^2)."""
    QQ = mask(2 * logQ)
    sp = [x & QQ for x in s]  # s mod Q^2, non-negative representatives
    as_ = negacyclic_mul(a, sp)
    ss = negacyclic_mul(sp, sp)
    Q = 1 << logQ
    bx = [(x + int(ei) + Q * y) & QQ for x, ei, y in zip(as_, e, ss)]
    return bx, [x & QQ for x in a]


def encrypt(t, s, a, e, logq: int):
    """A fresh ciphertext of plaintext t at level q: ax = a, bx = a s + e + t (mod q).

    (The secret-key form of the paper's encryption: the public key is
    (a s + e', a), whose products with u fold into a and e here.)"""
    qm = mask(logq)
    sp = [int(x) & qm for x in s]
    as_ = negacyclic_mul([x & qm for x in a], sp)
    bx = [(x + int(ei) + int(ti)) & qm for x, ei, ti in zip(as_, e, t)]
    return bx, [x & qm for x in a]


def decrypt(ct, s, logq: int) -> list:
    """t = bx - ax s (mod q), centred in [-q/2, q/2)."""
    qm = mask(logq)
    bx, ax = ct
    sp = [int(x) & qm for x in s]
    axs = negacyclic_mul(ax, sp)
    half = 1 << (logq - 1)
    return [(((b - x) & qm) ^ half) - half for b, x in zip(bx, axs)]


# ---------------------------------------------------------------- word arrays
def words_to_ints(w: np.ndarray) -> list:
    """[W][N] uint64 little-endian words -> N Python ints."""
    W, n = w.shape
    out = [0] * n
    for k in range(W - 1, -1, -1):
        col = w[k].tolist()
        out = [(o << 64) | c for o, c in zip(out, col)]
    return out


def ints_to_words(x, W: int) -> np.ndarray:
    """N non-negative Python ints < 2^(64 W) -> [W][N] uint64 words."""
    n = len(x)
    out = np.empty((W, n), dtype=np.uint64)
    m = mask(64)
    cur = list(x)
    for k in range(W):
        out[k] = np.array([c & m for c in cur], dtype=np.uint64)
        cur = [c >> 64 for c in cur]
    assert not any(cur)
    return out
