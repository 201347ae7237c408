"""Pins of the non-RNS (big-integer) HEAAN oracle against mathematics that
does not come from the oracle itself: schoolbook products over Z, monomial
shifts, the Karatsuba identity, exact rounding, and decryption of the
product within the key-switching error bound."""
import random

import numpy as np
import pytest

import synth
from oracle import heaan_bigint as hb


def _schoolbook_z(a, b):
    """Negacyclic product over Z, straight from X^N = -1."""
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += a[i] * b[j]
            else:
                c[k - n] -= a[i] * b[j]
    return c


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("bits", [1, 61, 64, 200, 1200])
def test_negacyclic_equals_schoolbook(n, bits):
    r = random.Random(n * 1000 + bits)
    for trial in range(3):
        if trial == 0:
            a = [(1 << bits) - 1] * n  # extreme: every coefficient maximal
            b = [(1 << bits) - 1] * n
        elif trial == 1:
            a = [0] * n
            b = [r.getrandbits(bits) for _ in range(n)]
        else:
            a = [r.getrandbits(bits) for _ in range(n)]
            b = [r.getrandbits(bits) for _ in range(n)]
        assert hb.negacyclic_mul(a, b) == _schoolbook_z(a, b)


def test_negacyclic_monomial_shift():
    """a * X^j rotates a by j with the wrapped part negated."""
    r = random.Random(5)
    n = 32
    a = [r.getrandbits(100) for _ in range(n)]
    for j in (0, 1, 7, 31):
        mono = [0] * n
        mono[j] = 1
        want = [(-a[k - j + n]) if k < j else a[k - j] for k in range(n)]
        assert hb.negacyclic_mul(a, mono) == want


def test_karatsuba_identity():
    """(ax1+bx1)(ax2+bx2) - ax1 ax2 - bx1 bx2 = ax1 bx2 + bx1 ax2 (mod q): the
    region-1 terms of HE Mul give the cross term of the tensor product."""
    r = random.Random(9)
    n, logq = 8, 90
    qm = hb.mask(logq)
    ax1, bx1, ax2, bx2 = ([r.getrandbits(logq) for _ in range(n)] for _ in range(4))
    ev = ([r.getrandbits(2 * logq) for _ in range(n)], [0] * n)  # evk.ax = 0: no key-switch term in ax3
    bx3, ax3 = hb.he_mul((bx1, ax1), (bx2, ax2), ev, logq, logq)
    cross = [(x + y) & qm for x, y in zip(_schoolbook_z(ax1, bx2), _schoolbook_z(bx1, ax2))]
    assert ax3 == cross
    bxbx = [c & qm for c in _schoolbook_z(bx1, bx2)]
    axax = [c & qm for c in _schoolbook_z(ax1, ax2)]
    # bx3 - bxbx is the key-switch term of evk.bx alone: round(axax*evk.bx / Q)
    ks = [(b - y) & qm for b, y in zip(bx3, bxbx)]
    prod = _schoolbook_z(axax, ev[0])
    Q = 1 << logq
    for k in range(n):
        v = prod[k] % (Q << logq)
        quo, rem = divmod(v, Q)
        assert ks[k] == (quo + (1 if 2 * rem >= Q else 0)) % (1 << logq)


def test_rescale_rounds_to_nearest():
    r = random.Random(11)
    logq, logp = 100, 30
    ct = ([r.getrandbits(logq) for _ in range(16)], [r.getrandbits(logq) for _ in range(16)])
    ct[0][0] = (1 << 29)          # exactly half: rounds up
    ct[0][1] = (1 << 29) - 1      # just below half: rounds down
    ct[0][2] = (1 << logq) - 1    # top value: wraps to 0 mod q/p
    out = hb.rescale(ct, logq, logp)
    p = 1 << logp
    for poly_in, poly_out in zip(ct, out):
        for x, y in zip(poly_in, poly_out):
            quo, rem = divmod(x, p)
            assert y == (quo + (2 * rem >= p)) % (1 << (logq - logp))
    assert out[0][0] == 1 and out[0][1] == 0 and out[0][2] == 0


def test_words_roundtrip():
    x = synth.uniform_bigint(3, 1200, 37)
    ints = hb.words_to_ints(x)
    assert max(ints).bit_length() <= 1200
    assert np.array_equal(hb.ints_to_words(ints, x.shape[0]), x)
    assert ints[5] == sum(int(x[k][5]) << (64 * k) for k in range(x.shape[0]))


def _small_secret(r, n, h):
    s = [0] * n
    for i in r.sample(range(n), h):
        s[i] = r.choice((-1, 1))
    return s


@pytest.mark.parametrize("n,logq,logQ", [(16, 120, 120), (16, 90, 120), (32, 200, 240)])
def test_he_mul_decrypts_to_product(n, logq, logQ):
    """decrypt(HE Mul(c1, c2)) = (t1 + e1)(t2 + e2) + axax e / Q + rounding,
    so it is within N (q/Q) max|e| + (1 + h)/2 of the exact product of the
    decrypted inputs -- a dropped term, a wrong sign or a swapped operand
    anywhere in the oracle's HE Mul leaves an error of order q instead."""
    r = random.Random(n + logq)
    h = 8
    s = _small_secret(r, n, h)
    e_evk = [r.randint(-19, 19) for _ in range(n)]
    evk = hb.evk_from_secret(s, [r.getrandbits(2 * logQ) for _ in range(n)], e_evk, logQ)
    cts, dec = [], []
    for _ in range(2):
        t = [r.randint(-(1 << 20), 1 << 20) for _ in range(n)]
        e = [r.randint(-19, 19) for _ in range(n)]
        ct = hb.encrypt(t, s, [r.getrandbits(logq) for _ in range(n)], e, logq)
        d = hb.decrypt(ct, s, logq)
        assert d == [a + b for a, b in zip(t, e)]  # encryption pin
        cts.append(ct)
        dec.append(d)
    c3 = hb.he_mul(cts[0], cts[1], evk, logq, logQ)
    got = hb.decrypt(c3, s, logq)
    want = _schoolbook_z(dec[0], dec[1])
    bound = n * (1 << logq) * 19 / (1 << logQ) + (1 + h) / 2 + 1
    err = max(abs(g - w) for g, w in zip(got, want))
    assert err <= bound, (err, bound)
    # a planted mistake (ax3 without the key-switch term) must be caught
    bad = (c3[0], [(a - k) & hb.mask(logq) for a, k in zip(c3[1], hb.key_switch_part(
        [c & hb.mask(logq) for c in hb.negacyclic_mul(cts[0][1], cts[1][1])], evk[1], logq, logQ))])
    err_bad = max(abs(g - w) for g, w in zip(hb.decrypt(bad, s, logq), want))
    assert err_bad > 1000 * bound


def test_rescale_decrypts_to_quotient():
    r = random.Random(21)
    n, logq, logp, h = 16, 120, 30, 8
    s = _small_secret(r, n, h)
    t = [r.randint(-(1 << 60), 1 << 60) for _ in range(n)]
    ct = hb.encrypt(t, s, [r.getrandbits(logq) for _ in range(n)], [0] * n, logq)
    got = hb.decrypt(hb.rescale(ct, logq, logp), s, logq - logp)
    for g, x in zip(got, t):
        assert abs(g - x / (1 << logp)) <= (1 + h) / 2 + 1


@pytest.mark.parametrize("sparse", [False, True])
def test_he_mul_at_equals_full_product(sparse):
    """The chosen-coefficient HE Mul (direct negacyclic sums per
    coefficient) equals the full Kronecker-product HE Mul at every index,
    with and without rescale, dense and sparse second operands, including
    maximal coefficients."""
    rng = random.Random(5 + sparse)
    n, logq, logQ, logp = 16, 200, 220, 30
    qm = hb.mask(logq)
    ct1 = ([rng.getrandbits(logq) for _ in range(n)], [rng.getrandbits(logq) for _ in range(n)])
    if sparse:
        ax2 = [0] * n
        bx2 = [0] * n
        for j in rng.sample(range(n), 3):
            ax2[j] = rng.getrandbits(logq)
        for j in rng.sample(range(n), 2):
            bx2[j] = qm  # maximal
        ct2 = (bx2, ax2)
    else:
        ct2 = ([rng.getrandbits(logq) for _ in range(n)], [qm] * n)
    evk = ([rng.getrandbits(2 * logQ) for _ in range(n)], [rng.getrandbits(2 * logQ) for _ in range(n)])
    full = hb.he_mul(ct1, ct2, evk, logq, logQ)
    idx = list(range(n))
    assert hb.he_mul_at(ct1, ct2, evk, logq, logQ, idx) == tuple(full)
    resc = hb.rescale(full, logq, logp)
    assert hb.he_mul_at(ct1, ct2, evk, logq, logQ, [0, 7, n - 1], logp) == tuple(
        [p[k] for k in (0, 7, n - 1)] for p in resc)
