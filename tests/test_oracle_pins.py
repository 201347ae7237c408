"""Pins of the CPU oracle against mathematics that does not come from the
oracle itself: brute force, closed forms, exact big-integer identities and
the paper's operation counts (Table IV)."""
import json
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers
def _sprp(n: int, bases) -> bool:
    """Independent strong-probable-prime test (Python ints)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in bases:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _trial_prime(n: int) -> bool:
    if n < 2:
        return False
    i = 2
    while i * i <= n:
        if n % i == 0:
            return False
        i += 1
    return True


def _tiny_ctx(log_n=4, L=5, K=2, dnum=3, qbits=50, pbits=60):
    used, q, p = [], [], []
    for _ in range(L):
        (x,) = oracle.gen_primes(log_n, qbits, 1, exclude=used)
        used.append(x)
        q.append(x)
    for _ in range(K):
        (x,) = oracle.gen_primes(log_n, pbits, 1, exclude=used)
        used.append(x)
        p.append(x)
    return oracle.Context(log_n, q, p, dnum)


def _coef(ctx, poly_limbs, basis_idx):
    """INTT each limb (limb r of poly_limbs is mod ctx.moduli[basis_idx[r]])."""
    return np.stack([ctx.intt(bi, poly_limbs[r]) for r, bi in enumerate(basis_idx)])


def _prod(xs):
    r = 1
    for x in xs:
        r *= int(x)
    return r


# ---------------------------------------------------------------- O0 primes
def test_is_prime_matches_trial_division():
    for n in list(range(0, 3000)) + [2**31 - 1, 2**31 + 11, 1000003 * 1000033]:
        assert oracle.is_prime(n) == _trial_prime(n) if n < 10**7 else oracle.is_prime(n) == _sprp(n, range(2, 60))


def test_gen_primes_small_bruteforce():
    # largest primes < 2^20 that are 1 mod 32, by brute force
    twoN = 32
    want = [x for x in range((1 << 20) - 1, 1, -1) if x % twoN == 1 and _trial_prime(x)][:6]
    assert oracle.gen_primes(4, 20, 6) == want


@pytest.mark.parametrize("wname", ["n12_L3", "n16_L24", "n17_L45", "n15_L12", "n16_L40_w30"])
def test_workload_primes_are_largest_and_distinct(wname):
    w = synth.WORKLOADS[wname]
    q, p = oracle.workload_primes(w)
    allp = q + p
    assert len(set(allp)) == len(allp) == w.L + w.K
    twoN = 2 * w.N
    rnd = random.Random(7)
    bases = [rnd.randrange(2, 2**40) for _ in range(8)]
    for x, b in zip(allp, list(w.q_bits) + [w.p_bits] * w.K):
        assert x % twoN == 1 and x < (1 << b) and x > (1 << (b - 1))
        assert _sprp(x, bases)
    # "largest first": no skipped candidate above each 60-bit prime and above
    # the smallest 50-bit prime is prime unless it is already in the list
    for b in set(w.q_bits) | {w.p_bits}:
        chosen = sorted([x for x, bb in zip(allp, list(w.q_bits) + [w.p_bits] * w.K) if bb == b])
        lo = chosen[0]
        x = ((1 << b) - 1) // twoN * twoN + 1
        while x > lo:
            if x not in chosen:
                assert not _sprp(x, bases), hex(x)
            x -= twoN


# ---------------------------------------------------------------- O1 root
@pytest.mark.parametrize("q,log_n", [(97, 3), (257, 6), (7681, 8), (12289, 9)])
def test_min_root_bruteforce(q, log_n):
    N = 1 << log_n
    roots = [x for x in range(1, q) if pow(x, N, q) == q - 1]
    assert len(roots) == N              # exactly the N primitive 2N-th roots
    assert oracle.min_root(q, log_n) == min(roots)


def test_psi_of_workload_primes_is_primitive():
    w = synth.CFG_N12
    ctx = oracle.Context.for_workload(w)
    for i, m in enumerate(ctx.moduli):
        psi = ctx.psi(i)
        assert pow(psi, w.N, m) == m - 1


# ---------------------------------------------------------------- O2 NTT
@pytest.mark.parametrize("log_n", [2, 4, 5])
def test_ntt_closed_form(log_n):
    ctx = _tiny_ctx(log_n=log_n)
    N = ctx.N
    rnd = np.random.default_rng(log_n)
    for idx in (0, ctx.L):           # a q-prime and a special prime
        m = ctx.moduli[idx]
        psi = ctx.psi(idx)
        a = rnd.integers(0, m, size=N, dtype=np.uint64)
        assert [int(x) for x in ctx.ntt(idx, a)] == oracle.ntt_closed_form(a, m, psi)
        one = np.zeros(N, dtype=np.uint64)
        one[0] = 1
        assert (ctx.ntt(idx, one) == 1).all()
        X = np.zeros(N, dtype=np.uint64)
        X[1] = 1
        want = [pow(psi, 2 * oracle.bitrev(i, log_n) + 1, m) for i in range(N)]
        assert [int(v) for v in ctx.ntt(idx, X)] == want
        assert pow(psi, N, m) == m - 1


@pytest.mark.parametrize("log_n", [2, 4, 6])
def test_ntt_product_equals_schoolbook(log_n):
    ctx = _tiny_ctx(log_n=log_n)
    N = ctx.N
    rnd = np.random.default_rng(100 + log_n)
    for idx in range(ctx.L + ctx.K):
        m = ctx.moduli[idx]
        cases = [rnd.integers(0, m, size=(2, N), dtype=np.uint64),
                 np.full((2, N), m - 1, dtype=np.uint64),
                 np.zeros((2, N), dtype=np.uint64)]
        for a, b in cases:
            prod = ctx.intt(idx, (np.array([int(x) * int(y) % m for x, y in zip(ctx.ntt(idx, a), ctx.ntt(idx, b))],
                                           dtype=np.uint64)))
            assert [int(v) for v in prod] == oracle.schoolbook_negacyclic(a, b, m)


@pytest.mark.parametrize("wname", ["n12_L3", "n15_L12", "n16_L24", "n17_L45", "n16_L40_w30"])
def test_ntt_roundtrip_identity(wname):
    w = synth.WORKLOADS[wname]
    q, p = oracle.workload_primes(w)
    ctx = oracle.Context(w.log_n, q[:2], p[:1], 1)
    for idx in range(3):
        a = synth.uniform_limbs(idx, [ctx.moduli[idx]], w.N)[0]
        assert (ctx.intt(idx, ctx.ntt(idx, a)) == a).all()
        assert (ctx.ntt(idx, ctx.intt(idx, a)) == a).all()


def test_power_table_is_powers_of_psi():
    ctx = _tiny_ctx(log_n=5)
    for idx in (0, ctx.L):
        m, psi = ctx.moduli[idx], ctx.psi(idx)
        pw = ctx.powers(idx)
        assert [int(x) for x in pw] == [pow(psi, k, m) for k in range(2 * ctx.N)]
        assert int(pw[ctx.N]) == m - 1


# ---------------------------------------------------------------- P9 op counts (Table IV)
def test_op_counts_match_table_iv():
    with open(os.path.join(GOLDEN, "table4_op_counts.json")) as f:
        g = json.load(f)
    ctx = _tiny_ctx(log_n=6)
    N, logN = ctx.N, 6
    a = np.arange(N, dtype=np.uint64)
    np_ = 3
    oracle.reset_counters()
    for idx in range(np_):
        ctx.ntt(idx, a)
    ntt_c, _ = oracle.counters()
    oracle.reset_counters()
    for idx in range(np_):
        ctx.intt(idx, a)
    _, intt_c = oracle.counters()
    env = {"N": N, "logN": logN, "np": np_}
    assert ntt_c == eval(g["NTT"]["modmul"], {}, env)
    assert intt_c == eval(g["iNTT"]["modmul"], {}, env)


# ---------------------------------------------------------------- O6 / P8 tensor
def test_tensor_equals_karatsuba_and_definition():
    ctx = _tiny_ctx(log_n=4)
    lv = 4
    ct1 = synth.random_ciphertext(1, ctx.q[:lv], ctx.N)
    ct2 = synth.random_ciphertext(2, ctx.q[:lv], ctx.N)
    d = ctx.tensor(lv, ct1, ct2)
    for i in range(lv):
        m = ctx.q[i]
        for k in range(ctx.N):
            b1, a1, b2, a2 = (int(ct1[0, i, k]), int(ct1[1, i, k]), int(ct2[0, i, k]), int(ct2[1, i, k]))
            kara = ((a1 + b1) * (a2 + b2) - b1 * b2 - a1 * a2) % m
            assert int(d[0, i, k]) == b1 * b2 % m
            assert int(d[1, i, k]) == kara == (a1 * b2 + a2 * b1) % m
            assert int(d[2, i, k]) == a1 * a2 % m


# ---------------------------------------------------------------- O7 / P4 ModUp
@pytest.mark.parametrize("level", [5, 4, 1])
def test_modup_fast_conversion_identity(level):
    """Fast conversion without overflow correction: with X the exact CRT
    value of the digit's coefficients and y_i = x_i [(Qt/q_i)^-1]_{q_i},
    every target limb holds X + u Qt with u = floor(sum_i y_i / q_i), the
    overflow count of the matrix form of an iCRT followed at once by a CRT
    (Table XI, Algorithm 6); u is computed here from Python integers, and an exact
    conversion (u = 0 everywhere) fails the check."""
    ctx = _tiny_ctx(log_n=4, L=5, K=2, dnum=3)
    d2 = synth.uniform_limbs(9, ctx.q[:level], ctx.N)
    dt = ctx.modup(level, d2)
    ext = list(range(level)) + [ctx.L + k for k in range(ctx.K)]
    x = _coef(ctx, d2, list(range(level)))
    overflow_seen = False
    for j in range(ctx.num_digits(level)):
        D = ctx.digit(j, level)
        Qt = _prod(ctx.q[i] for i in D)
        X = oracle.crt([x[i] for i in D], [ctx.q[i] for i in D])
        z = _coef(ctx, dt[j], ext)
        for e, bi in enumerate(ext):
            if e in D:
                assert (dt[j][e] == d2[e]).all()     # own limbs copied in NTT form
        for k in range(ctx.N):
            # y_i in [0, q_i); sum_i y_i Qt/q_i = X + u Qt exactly
            ys = [int(x[i][k]) * pow(Qt // ctx.q[i] % ctx.q[i], -1, ctx.q[i]) % ctx.q[i] for i in D]
            u = sum(F * (Qt // ctx.q[i]) for F, i in zip(ys, D)) // Qt
            assert sum(Fraction(F, ctx.q[i]) for F, i in zip(ys, D)) // 1 == u   # = floor(sum y_i / q_i)
            assert 0 <= u < len(D)
            overflow_seen |= u > 0
            for e, bi in enumerate(ext):
                if e not in D:
                    assert int(z[e][k]) == (X[k] + u * Qt) % ctx.moduli[bi], (j, k, e)
    if level > 1:
        assert overflow_seen    # the reading "no overflow correction" is visible


def test_modup_alpha1_is_plain_reduction():
    # one prime per digit: the conversion is x mod t exactly
    ctx = _tiny_ctx(log_n=4, L=3, K=1, dnum=3)
    d2 = synth.uniform_limbs(3, ctx.q, ctx.N)
    dt = ctx.modup(3, d2)
    ext = [0, 1, 2, ctx.L]
    x = _coef(ctx, d2, [0, 1, 2])
    for j in range(3):
        z = _coef(ctx, dt[j], ext)
        for e, bi in enumerate(ext):
            if e != j:
                assert [int(v) for v in z[e]] == [int(v) % ctx.moduli[bi] for v in x[j]]


# ---------------------------------------------------------------- O9 / P5 ModDown
@pytest.mark.parametrize("K", [1, 2])
def test_moddown_floor_identity(K):
    """ModDown and the combine with the tensor terms: out_u = d_u + ModDown(ks_u)
    with ModDown(X) = floor(X / P) - v, v in [0, K) (exactly floor(X / P)
    when K = 1), for nonzero d so the combine's sign and operand are pinned."""
    ctx = _tiny_ctx(log_n=4, L=4, K=K, dnum=2)
    level = 4
    ext = list(range(level)) + [ctx.L + k for k in range(K)]
    ks = np.stack([synth.uniform_limbs(20 + u, [ctx.moduli[b] for b in ext], ctx.N) for u in range(2)])
    d = np.stack([synth.uniform_limbs(40 + u, ctx.q[:level], ctx.N) for u in range(3)])
    out = ctx.moddown_combine(level, ks, d)
    P = _prod(ctx.p)
    QP = _prod(ctx.q[:level]) * P
    Ql = _prod(ctx.q[:level])
    vs_seen = set()
    for u in range(2):
        X = oracle.crt(_coef(ctx, ks[u], ext), [ctx.moduli[b] for b in ext])
        D = oracle.crt(_coef(ctx, d[u], list(range(level))), ctx.q[:level])
        o = oracle.crt(_coef(ctx, out[u], list(range(level))), ctx.q[:level])
        for k in range(ctx.N):
            assert 0 <= X[k] < QP and D[k] != 0
            vs = [v for v in range(K) if (D[k] + X[k] // P - v) % Ql == o[k]]
            assert len(vs) == 1
            vs_seen.add(vs[0])
            if K == 1:
                assert o[k] == (D[k] + X[k] // P) % Ql
    assert vs_seen <= set(range(K))


# ---------------------------------------------------------------- O10 / P6 rescale
@pytest.mark.parametrize("level", [2, 3, 5])
def test_rescale_is_exact_rounding(level):
    ctx = _tiny_ctx(log_n=4, L=5, K=2, dnum=3)
    ct = synth.random_ciphertext(31 + level, ctx.q[:level], ctx.N)
    out = ctx.rescale(level, ct)
    ql = ctx.q[level - 1]
    Qlm = _prod(ctx.q[:level - 1])
    for u in range(2):
        C = oracle.crt(_coef(ctx, ct[u], list(range(level))), ctx.q[:level])
        o = oracle.crt(_coef(ctx, out[u], list(range(level - 1))), ctx.q[:level - 1])
        for k in range(ctx.N):
            rnd = (2 * C[k] + ql) // (2 * ql)     # round(C / ql), ql odd so no ties
            assert o[k] == rnd % Qlm


# ---------------------------------------------------------------- O4 / O8 / P7 key switch
def _keys(ctx, w_like_h=4, seed=1):
    N = ctx.N
    s = synth.ternary_hwt(seed, N, w_like_h)
    e_pk = synth.gaussian(seed, N, 13)[0]
    e_evk = synth.gaussian(seed, N, 14, ctx.dnum)
    a_pk = synth.uniform_limbs(seed, ctx.q, N, 30)
    a_evk = np.stack([synth.uniform_limbs(seed, ctx.moduli, N, 40 + j) for j in range(ctx.dnum)])
    pk, evk = ctx.keygen(s, e_pk, e_evk, a_pk, a_evk)
    return s, pk, evk


def _negacyclic_int(a, b):
    N = len(a)
    c = [0] * N
    for i in range(N):
        if a[i] == 0:
            continue
        for j in range(N):
            k = i + j
            if k < N:
                c[k] += a[i] * b[j]
            else:
                c[k - N] -= a[i] * b[j]
    return c


@pytest.mark.parametrize("level", [5, 3])
def test_keyswitch_correctness_bound(level):
    ctx = _tiny_ctx(log_n=5, L=5, K=2, dnum=3)
    h = 4
    s, pk, evk = _keys(ctx, h)
    d2 = synth.uniform_limbs(77, ctx.q[:level], ctx.N)
    dt = ctx.modup(level, d2)
    ks = ctx.inner_product(level, dt, evk)
    out = ctx.moddown_combine(level, ks, np.zeros((3, level, ctx.N), dtype=np.uint64))
    Ql = _prod(ctx.q[:level])
    ob = oracle.crt_centered(_coef(ctx, out[0], list(range(level))), ctx.q[:level])
    oa = oracle.crt_centered(_coef(ctx, out[1], list(range(level))), ctx.q[:level])
    D2 = oracle.crt(_coef(ctx, d2, list(range(level))), ctx.q[:level])
    sl = [int(v) for v in s]
    s2 = _negacyclic_int(sl, sl)
    want = _negacyclic_int(s2, D2)
    got = [x - y for x, y in zip(ob, _negacyclic_int(sl, oa))]
    P = _prod(ctx.p)
    maxQt = max(_prod(ctx.q[i] for i in ctx.digit(j, level)) for j in range(ctx.num_digits(level)))
    bound = (ctx.K + 1) * (1 + h) + ctx.dnum * ctx.N * ctx.alpha * (maxQt / P) * 6 * synth.SIGMA
    for k in range(ctx.N):
        diff = (got[k] - want[k]) % Ql
        diff = diff - Ql if 2 * diff >= Ql else diff
        assert abs(diff) <= bound, (k, diff, bound)


# ---------------------------------------------------------------- O5 encoding
def test_encode_matches_definition_small():
    N = 16
    z = synth.unit_disk(5, N // 2)
    scale = 2.0**20
    m = oracle.encode(z, scale, N)
    zeta = np.exp(1j * np.pi / N)
    ex = oracle.slot_exponents(N)
    direct = [round((2.0 / N) * np.real(sum(scale * z[j] * zeta ** (-int(ex[j]) * k) for j in range(N // 2))))
              for k in range(N)]
    assert list(m) == direct
    back = oracle.decode([int(v) for v in m], scale)
    assert np.max(np.abs(back - z)) < N / scale


def test_encode_decode_roundtrip_n12():
    N = 1 << 12
    z = synth.unit_disk(2, N // 2)
    m = oracle.encode(z, 2.0**40, N)
    back = oracle.decode([int(v) for v in m], 2.0**40)
    assert np.max(np.abs(back - z)) < 2.0**-25


# ---------------------------------------------------------------- O11 FP64 gate on the oracle
def _fresh_pair(ctx, w, level):
    kd = synth.key_draws(w)
    a_pk = synth.uniform_limbs(synth.SEED_KEYS, ctx.q, w.N, 30)
    a_evk = np.stack([synth.uniform_limbs(synth.SEED_KEYS, ctx.moduli, w.N, 40 + j) for j in range(w.dnum)])
    pk, evk = ctx.keygen(kd.s, kd.e_pk, kd.e_evk, a_pk, a_evk)
    za, zb = synth.unit_disk(synth.SEED_MSG_A, w.slots), synth.unit_disk(synth.SEED_MSG_B, w.slots)
    scale = 2.0**w.log_scale
    cts = []
    for z, seed in ((za, synth.SEED_ENC_A), (zb, synth.SEED_ENC_B)):
        ed = synth.enc_draws(w, seed)
        cts.append(ctx.encrypt(level, oracle.encode(z, scale, w.N), ed.v, ed.e0, ed.e1, pk))
    return kd.s, evk, za, zb, cts


def test_decrypt_of_he_mul_matches_fp64_product_n12():
    w = synth.CFG_N12
    ctx = oracle.Context.for_workload(w)
    level = w.L
    s, evk, za, zb, (c1, c2) = _fresh_pair(ctx, w, level)
    scale = 2.0**w.log_scale
    # fresh ciphertexts decrypt to the messages
    assert np.max(np.abs(ctx.decrypt(level, c1, s, scale) - za)) < 2.0**-20
    relin, out = ctx.he_mul(level, c1, c2, evk)
    want = za * zb
    got_pre = ctx.decrypt(level, relin, s, scale * scale)
    rel_pre = np.linalg.norm(got_pre - want) / np.linalg.norm(want)
    got = ctx.decrypt(level - 1, out, s, scale * scale / ctx.q[level - 1])
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel_pre < 2.0**-20, rel_pre
    assert rel < 2.0**-20, rel


def test_he_add_decrypts_to_sum_n12():
    """HE Add (Sec. III-B) is linear under decryption: the decrypted sum is
    the sum of the decrypted inputs, exactly, modulo each q_i."""
    w = synth.CFG_N12
    ctx = oracle.Context.for_workload(w)
    level = w.L
    s, evk, za, zb, (c1, c2) = _fresh_pair(ctx, w, level)
    c3 = ctx.he_add(level, c1, c2)
    d1, d2, d3 = (ctx.decrypt_limbs(level, c, s) for c in (c1, c2, c3))
    for i, q in enumerate(ctx.q[:level]):
        assert np.array_equal((d1[i].astype(object) + d2[i].astype(object)) % q, d3[i].astype(object))
    scale = 2.0**w.log_scale
    assert np.max(np.abs(ctx.decrypt(level, c3, s, scale) - (za + zb))) < 2.0**-19
    # wrap-around: every residue q-1 plus 1 gives 0
    ones = np.ones_like(c1)
    top = np.stack([np.stack([np.full(w.N, q - 1, dtype=np.uint64) for q in ctx.q[:level]])] * 2)
    assert not ctx.he_add(level, top, ones).any()


# ---------------------------------------------------------------- rotation (automorphisms)
def test_automorphism_closed_form_and_composition():
    """sigma_g(X) = X^g (negated past degree N), sigma_g1 sigma_g2 = sigma_(g1 g2),
    and sigma_g is a ring map: sigma(a b) = sigma(a) sigma(b)."""
    w = synth.CFG_TINY
    ctx = oracle.Context.for_workload(w)
    N, level = w.N, w.L
    mono = np.zeros((2, level, N), dtype=np.uint64)
    for i in range(level):
        x = np.zeros(N, dtype=np.uint64)
        x[1] = 1
        mono[0, i] = mono[1, i] = ctx.ntt(i, x)
    for g in (3, 5, 2 * N - 1, 25 % (2 * N)):
        out = ctx.automorphism(level, mono, g)
        for i in range(level):
            want = np.zeros(N, dtype=np.uint64)
            e = g % (2 * N)
            if e < N:
                want[e] = 1
            else:
                want[e - N] = ctx.q[i] - 1
            assert np.array_equal(ctx.intt(i, out[0, i]), want), (g, i)
    a = synth.random_ciphertext(3, ctx.q[:level], N)
    b = synth.random_ciphertext(4, ctx.q[:level], N)
    g1, g2 = 5, 2 * N - 5
    assert np.array_equal(ctx.automorphism(level, ctx.automorphism(level, a, g2), g1),
                          ctx.automorphism(level, a, (g1 * g2) % (2 * N)))
    prod = np.stack([np.stack([(a[u, i].astype(object) * b[u, i].astype(object) % ctx.q[i]).astype(np.uint64)
                               for i in range(level)]) for u in range(2)])
    sa, sb, sp = (ctx.automorphism(level, x, g1) for x in (a, b, prod))
    for u in range(2):
        for i in range(level):
            assert np.array_equal((sa[u, i].astype(object) * sb[u, i].astype(object) % ctx.q[i]).astype(np.uint64),
                                  sp[u, i])


@pytest.mark.parametrize("r", [1, 7, 1023])
def test_rotation_decrypts_to_rotated_slots_n12(r):
    """decrypt(rotate_r(enc(z))) ~ z shifted left by r slots (slot j <- j + r)
    within the key-switching error; the wrong rotation key misses by O(1)."""
    w = synth.CFG_N12
    ctx = oracle.Context.for_workload(w)
    level = w.L
    s, evk, za, zb, (c1, c2) = _fresh_pair(ctx, w, level)
    g = ctx.galois(r)
    e_rk = synth.gaussian(90 + r, w.N, 16, w.dnum)
    a_rk = np.stack([synth.uniform_limbs(91 + r, ctx.moduli, w.N, j) for j in range(w.dnum)])
    rk = ctx.keygen_rot(s, g, e_rk, a_rk)
    out = ctx.rotate(level, c1, rk, g)
    scale = 2.0**w.log_scale
    got = ctx.decrypt(level, out, s, scale)
    want = np.roll(za, -r)
    assert np.max(np.abs(got - want)) < 2.0**-20
    wrong = ctx.rotate(level, c1, ctx.keygen_rot(s, ctx.galois(r + 1), e_rk, a_rk), g)
    assert np.max(np.abs(ctx.decrypt(level, wrong, s, scale) - want)) > 2.0**-4


def test_decrypt_of_he_mul_w30_primes():
    """The 30-bit-prime variant (the paper's GPU word size): decrypt(HE Mul)
    matches the FP64 product of the slots, before and after the rescale."""
    w = synth.CFG_N16_W30
    ctx = oracle.Context.for_workload(w)
    level = 6
    s, evk, za, zb, (c1, c2) = _fresh_pair(ctx, w, level)
    scale = 2.0**w.log_scale
    relin, out = ctx.he_mul(level, c1, c2, evk)
    want = za * zb
    got_pre = ctx.decrypt(level, relin, s, scale * scale)
    got = ctx.decrypt(level - 1, out, s, scale * scale / ctx.q[level - 1])
    # scale 2^30: fresh noise ~ sqrt(N h) sigma per slot, i.e. about 2^-13
    # relative after the product; a wrong term errs by O(1)
    assert np.linalg.norm(got_pre - want) / np.linalg.norm(want) < 2.0**-10
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 2.0**-10



@pytest.mark.parametrize("wname", ["n12_L6_d1", "n12_L6_d6"])
def test_decrypt_of_he_mul_dnum_variants(wname):
    """Key switching with one digit (P > Q, the paper's evaluation key) and
    with one digit per prime: decrypt(HE Mul) matches the FP64 product."""
    w = synth.WORKLOADS[wname]
    ctx = oracle.Context.for_workload(w)
    level = w.L
    s, evk, za, zb, (c1, c2) = _fresh_pair(ctx, w, level)
    scale = 2.0**w.log_scale
    relin, out = ctx.he_mul(level, c1, c2, evk)
    want = za * zb
    got_pre = ctx.decrypt(level, relin, s, scale * scale)
    got = ctx.decrypt(level - 1, out, s, scale * scale / ctx.q[level - 1])
    assert np.linalg.norm(got_pre - want) / np.linalg.norm(want) < 2.0**-20
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 2.0**-20
