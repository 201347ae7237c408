"""GPU parity of the paper's non-RNS HE Mul (big-integer coefficients,
power-of-two moduli) against the big-integer oracle, through the C ABI."""
import functools

import numpy as np
import pytest

import synth
from oracle import heaan_bigint as hb
from gpu_common import log, need_gpu

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def big_ctx(log_n, logQ):
    P = need_gpu()
    return P.BigContext(log_n, logQ)


def _ints(arr):
    return [hb.words_to_ints(arr[u]) for u in range(arr.shape[0])]


@functools.lru_cache(maxsize=None)
def _oracle_case(log_n, logQ, logq, seed, kind):
    n = 1 << log_n
    W = synth.big_words(logQ)
    if kind == "random":
        c1 = synth.big_ciphertext(seed, logq, n, W)
        c2 = synth.big_ciphertext(seed + 1, logq, n, W)
    else:  # every coefficient q - 1: the largest products, Karatsuba sums wrap
        c1 = np.zeros((2, W, n), dtype=np.uint64)
        full = np.array([hb.mask(64)], dtype=np.uint64)
        for w in range(W):
            lo = 64 * w
            if lo + 64 <= logq:
                c1[:, w] = full
            elif lo < logq:
                c1[:, w] = np.uint64(hb.mask(logq - lo))
        c2 = c1.copy()
    ev = synth.big_evk(seed + 2, logQ, n)
    t1, t2, te = _ints(c1), _ints(c2), _ints(ev)
    log("oracle big he_mul", log_n, logQ, logq, kind)
    c3 = hb.he_mul(t1, t2, te, logq, logQ)
    return c1, c2, ev, c3


@pytest.mark.parametrize("logQ,logq,kind", [
    (300, 300, "random"),
    (300, 263, "random"),      # log q not a multiple of 32; log Q shift unaligned to 64
    (300, 300, "max"),
    (100, 71, "random"),
    (1200, 1200, "random"),    # the paper's log Q at N = 2^12
])
def test_big_mul_matches_oracle(logQ, logq, kind):
    _big_case(12, logQ, logq, kind)


def test_big_mul_other_ring():
    """N = 2^13 (another transform size, twice the coefficients per launch)."""
    _big_case(13, 300, 277, "random")


def _big_case(log_n, logQ, logq, kind):
    lib = big_ctx(log_n, logQ)
    c1, c2, ev, c3 = _oracle_case(log_n, logQ, logq, 7, kind)
    W = lib.W
    d1, d2 = lib.to_device(c1), lib.to_device(c2)
    evk_ntt = lib.evk_prepare(lib.to_device(ev))
    for logp in (0, 30):
        log("gpu big he_mul", logQ, logq, kind, "logp", logp)
        got = lib.to_host(lib.he_mul(logq, d1, d2, evk_ntt, logp=logp))
        want = hb.rescale(c3, logq, logp) if logp else c3
        for u in range(2):
            assert np.array_equal(got[u], hb.ints_to_words(want[u], W)), (logQ, logq, kind, logp, u)


def _sparse_mul(a, s_idx, s_val, n):
    """a * s for a ternary s with support s_idx (negacyclic, over Z)."""
    out = [0] * n
    for j, v in zip(s_idx, s_val):
        for k in range(n):
            x = a[k] * v
            if k + j < n:
                out[k + j] += x
            else:
                out[k + j - n] -= x
    return out


def test_big_mul_decrypts_at_full_size():
    """N = 2^16, log Q = 1200 (the paper's parameters): a real evaluation key
    and encryptions of sparse messages under a sparse secret; the decrypted
    product and its rescale are within the key-switching error bound of the
    exact product of the messages (a property that holds at any size)."""
    log_n, logQ, logq, logp, h = 16, 1200, 1200, 30, 32
    n = 1 << log_n
    lib = big_ctx(log_n, logQ)
    g = synth.rng(77)
    s_idx = [int(x) for x in g.choice(n, size=h, replace=False)]
    s_val = [int(x) for x in g.choice([-1, 1], size=h)]
    e_evk = [int(x) for x in synth.gaussian(78, n, 1)[0]]
    a_evk = hb.words_to_ints(synth.uniform_bigint(79, 2 * logQ, n))
    QQ = hb.mask(2 * logQ)
    log("full-size keys")
    as_ = _sparse_mul(a_evk, s_idx, s_val, n)
    s_poly = [0] * n
    for j, v in zip(s_idx, s_val):
        s_poly[j] = v
    ss = _sparse_mul(s_poly, s_idx, s_val, n)
    evk_bx = [(x + e + (y << logQ)) & QQ for x, e, y in zip(as_, e_evk, ss)]
    ev = np.stack([hb.ints_to_words(evk_bx, lib.W2), hb.ints_to_words(a_evk, lib.W2)])
    qm = hb.mask(logq)
    msgs, cts = [], []
    for k in range(2):
        t = [0] * n
        for j in g.choice(n, size=8, replace=False):
            t[int(j)] = int(g.integers(-(1 << 40), 1 << 40))
        a = hb.words_to_ints(synth.uniform_bigint(80 + k, logq, n))
        bx = [(x + y) & qm for x, y in zip(_sparse_mul(a, s_idx, s_val, n), t)]
        msgs.append(t)
        cts.append(np.stack([hb.ints_to_words(bx, lib.W), hb.ints_to_words(a, lib.W)]))
    evk_ntt = lib.evk_prepare(lib.to_device(ev))
    d1, d2 = lib.to_device(cts[0]), lib.to_device(cts[1])
    want = [0] * n
    nz1 = [(j, v) for j, v in enumerate(msgs[0]) if v]
    nz2 = [(j, v) for j, v in enumerate(msgs[1]) if v]
    for i, x in nz1:
        for j, y in nz2:
            if i + j < n:
                want[i + j] += x * y
            else:
                want[i + j - n] -= x * y
    bound = n * 19.2 * 2.0 ** (logq - logQ) + (1 + h) / 2 + 1
    for lp in (0, logp):
        log("full-size gpu he_mul logp", lp)
        out = lib.to_host(lib.he_mul(logq, d1, d2, evk_ntt, logp=lp))
        bx3, ax3 = _ints(out)
        lq = logq - lp
        m = hb.mask(lq)
        half = 1 << (lq - 1)
        axs = _sparse_mul(ax3, s_idx, s_val, n)
        dec = [(((b - x) & m) ^ half) - half for b, x in zip(bx3, axs)]
        scale = 1 << lp
        # exact integers: |dec * 2^lp - want| <= lim * 2^lp
        err = max(abs(d * scale - w) for d, w in zip(dec, want))
        lim = bound / scale + ((1 + h) / 2 + 1 if lp else 0)
        log("max error x 2^%d:" % lp, err, "bound", lim)
        assert err <= lim * scale


def test_big_errors():
    P = need_gpu()
    lib = big_ctx(12, 300)
    c = lib.empty(2, lib.W, lib.N)
    ev = lib.evk_prepare(lib.empty(2, lib.W2, lib.N).zero_())
    with pytest.raises(P.HeError):
        lib.he_mul(301, c, c, ev)            # log q above log Q
    with pytest.raises(P.HeError):
        lib.he_mul(0, c, c, ev)
    with pytest.raises(P.HeError):
        lib.he_mul(40, c, c, ev, logp=40)     # log p must be below log q
    with pytest.raises(P.HeError):
        lib.he_mul(300, c, c, ev, out=c)      # output aliases an input
    with pytest.raises(P.HeError):
        lib.he_mul(300, c, c, ev, ws=lib.empty(8))
    with pytest.raises(P.HeError):
        P.BigContext(12, 1300)                # beyond the supported log Q


@pytest.mark.parametrize("logq", [1200, 1111])
def test_big_mul_full_size_chosen_coefficients_bit_exact(logq):
    """The paper's parameters (N = 2^16, log Q = 1200; Table III, Table VII):
    ct1 and the evaluation key uniform and dense, ct2 with four nonzero
    coefficients per polynomial, so the oracle computes chosen output
    coefficients exactly (direct negacyclic sums: O(nnz) for the region-1
    products, one sum of N products per key-switched coefficient).  The
    GPU's output words at those coefficients -- ends, wrap positions next to
    ct2's support, random ones -- equal the oracle's bit for bit, with and
    without rescale (log p = 30); log q = 1111 is not a multiple of 32."""
    log_n, logQ = 16, 1200
    n = 1 << log_n
    lib = big_ctx(log_n, logQ)
    W = lib.W
    g = synth.rng(88 + logq)
    c1 = synth.big_ciphertext(90 + logq, logq, n, W)
    c2 = np.zeros((2, W, n), dtype=np.uint64)
    supp = {}
    for u in range(2):
        idx = sorted(int(x) for x in g.choice(n, size=4, replace=False))
        vals = synth.uniform_bigint(91 + logq + u, logq, 4, 0, W)
        c2[u][:, idx] = vals
        supp[u] = idx
    ev = synth.big_evk(92 + logq, logQ, n)
    chosen = sorted({0, 1, 2, n - 2, n - 1} | {(j + d) % n for u in supp for j in supp[u] for d in (-1, 0, 1)}
                    | {int(x) for x in g.integers(0, n, size=6)})
    log("chosen coefficients", len(chosen))
    t1, t2, te = _ints(c1), _ints(c2), _ints(ev)
    d1, d2 = lib.to_device(c1), lib.to_device(c2)
    evk_ntt = lib.evk_prepare(lib.to_device(ev))
    exact = hb.he_mul_at(t1, t2, te, logq, logQ, chosen)
    for logp in (0, 30):
        want = hb.rescale(exact, logq, logp) if logp else exact
        got = lib.to_host(lib.he_mul(logq, d1, d2, evk_ntt, logp=logp))
        for u in range(2):
            want_w = hb.ints_to_words(want[u], W)
            assert np.array_equal(got[u][:, chosen], want_w), (logq, logp, u)
        log("full size chosen coefficients bit-exact", logq, logp)
