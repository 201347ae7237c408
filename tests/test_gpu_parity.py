"""GPU parity: the HIP library (through its C ABI) against the CPU oracle,
element by element, on the same seeded inputs.  Integer results must be
bit-exact."""
import numpy as np
import pytest

import synth
from gpu_common import contexts, log, need_gpu, random_evk

pytestmark = pytest.mark.gpu

SMALL = synth.Workload("n12_L7_ragged", 12, 7, 3, 3, (60, 50, 50, 50, 50, 50, 50), 60, 64, 40)


@pytest.mark.parametrize("wname", ["n12_L3", "n13_L4", "n14_L6", "n15_L12", "n16_L24", "n17_L45"])
def test_ntt_intt_bit_exact(wname):
    lib, orc = contexts(wname)
    log("ntt", wname)
    idxs = [0, 1, lib.L - 1, lib.L, lib.L + lib.K - 1]
    for idx in idxs:
        a = synth.uniform_limbs(100 + idx, [orc.moduli[idx]], orc.N)[0]
        d = lib.to_device(a)
        lib.ntt(d, idx, inverse=False)
        got = lib.to_host(d)
        assert np.array_equal(got, orc.ntt(idx, a)), idx
        lib.ntt(d, idx, inverse=True)
        assert np.array_equal(lib.to_host(d), a), idx
        d2 = lib.to_device(a)
        lib.ntt(d2, idx, inverse=True)
        assert np.array_equal(lib.to_host(d2), orc.intt(idx, a)), idx


def test_ntt_extreme_values():
    lib, orc = contexts("n16_L24")
    for idx in (0, 5, lib.L):
        m = orc.moduli[idx]
        for a in (np.full(orc.N, m - 1, dtype=np.uint64), np.zeros(orc.N, dtype=np.uint64)):
            d = lib.to_device(a)
            lib.ntt(d, idx)
            assert np.array_equal(lib.to_host(d), orc.ntt(idx, a))


def _he_mul_case(w, level, seed=1):
    lib, orc = contexts(w)
    log("he_mul", getattr(w, "name", w), "level", level)
    ct1 = synth.random_ciphertext(seed, orc.q[:level], orc.N)
    ct2 = synth.random_ciphertext(seed + 1, orc.q[:level], orc.N)
    evk = random_evk(orc, 10 + seed)
    want_relin, want_out = orc.he_mul(level, ct1, ct2, evk, rescale=level >= 2)
    d1, d2, de = lib.to_device(ct1), lib.to_device(ct2), lib.to_device(evk)
    relin, out = lib.he_mul(level, d1, d2, de, relin=True, rescale=level >= 2)
    assert np.array_equal(lib.to_host(relin), want_relin)
    if level >= 2:
        assert np.array_equal(lib.to_host(out), want_out)
        # he_rescale alone
        assert np.array_equal(lib.to_host(lib.rescale(level, relin)), want_out)
        # rescaled output only (the relinearized ciphertext never written)
        _, out_only = lib.he_mul(level, d1, d2, de, relin=False, rescale=True)
        assert np.array_equal(lib.to_host(out_only), want_out)
        # relinearized output only
        relin_only, none = lib.he_mul(level, d1, d2, de, relin=True, rescale=False)
        assert none is None
        assert np.array_equal(lib.to_host(relin_only), want_relin)


@pytest.mark.parametrize("level", [3, 2, 1])
def test_he_mul_n12(level):
    _he_mul_case("n12_L3", level)


@pytest.mark.parametrize("level", [7, 6, 4, 3, 1])
def test_he_mul_ragged_digits(level):
    _he_mul_case(SMALL, level)


@pytest.mark.parametrize("level", [24, 17, 9, 4])
def test_he_mul_n16(level):
    _he_mul_case("n16_L24", level)


@pytest.mark.parametrize("level", [12, 5])
def test_he_mul_n15(level):
    _he_mul_case("n15_L12", level)


@pytest.mark.parametrize("level", [45, 31])
def test_he_mul_n17(level):
    _he_mul_case("n17_L45", level)


@pytest.mark.parametrize("wname,level", [("n16_L24_d1", 24), ("n16_L24_d1", 9), ("n16_L24_d24", 24),
                                         ("n16_L24_d24", 5), ("n12_L6_d1", 6), ("n12_L6_d6", 6),
                                         ("n12_L28_d1", 28), ("n12_L28_d1", 13)])
def test_he_mul_dnum_variants(wname, level):
    """Key switching with dnum = 1 (one digit of up to 24 primes, 21 special
    primes: the conversion's runs of 15 sources folded in 128 bits; 28 and
    24 sources at N = 2^12, the conversion's widest source bound, with the
    digit cut to 13 primes at level 13) and dnum = L (one prime per digit,
    24 digits in the inner product)."""
    _he_mul_case(wname, level)


@pytest.mark.parametrize("wname,level", [("n13_L4", 4), ("n13_L4", 3), ("n14_L6", 6), ("n14_L6", 2)])
def test_he_mul_n13_n14(wname, level):
    """Ring degrees 2^13 and 2^14: 128-point blocks sub-transforms (and
    64- / 128-point cols sub-transforms) in every pass, including the inner
    product's inverse blocks epilogue."""
    _he_mul_case(wname, level)


@pytest.mark.parametrize("level", [40, 11, 2])
def test_he_mul_w30_primes(level):
    """The paper's GPU word size: 40 primes of 30 bits (log Q = 1200)."""
    _he_mul_case("n16_L40_w30", level)


def test_he_mul_extreme_inputs():
    lib, orc = contexts("n16_L24")
    level = 24
    ct1 = np.stack([np.stack([np.full(orc.N, q - 1, dtype=np.uint64) for q in orc.q[:level]])] * 2)
    ct2 = ct1.copy()
    evk = np.stack([np.stack([np.stack([np.full(orc.N, m - 1, dtype=np.uint64) for m in orc.moduli])] * 2)]
                   * orc.dnum)
    want_relin, want_out = orc.he_mul(level, ct1, ct2, evk)
    relin, out = lib.he_mul(level, lib.to_device(ct1), lib.to_device(ct2), lib.to_device(evk))
    assert np.array_equal(lib.to_host(relin), want_relin)
    assert np.array_equal(lib.to_host(out), want_out)


def test_he_mul_maximal_modup_sources():
    """Every mod-up source residue at its maximum q_i - 1, so the conversion's
    128-bit sums reach their largest values: with ct2's a the NTT of the
    polynomial 1, d2 = ct1's a, chosen as the NTT of the constant coefficient
    vector v_i = (q_i - 1) [Q~_j / q_i]_{q_i}; the conversion's per-limb factor
    [(Q~_j / q_i)^-1]_{q_i} turns every coefficient into q_i - 1."""
    lib, orc = contexts("n16_L24")
    level = 24
    log("he_mul maximal mod-up sources", level)
    rng = np.random.default_rng(31)
    a1, a2 = [], []
    for j in range(orc.num_digits(level)):
        dig = [int(orc.q[i]) for i in orc.digit(j, level)]
        qt = 1
        for q in dig:
            qt *= q
        for q in dig:
            v = (q - 1) * ((qt // q) % q) % q
            limb = orc.ntt(len(a1), np.full(orc.N, v, dtype=np.uint64))
            assert np.all(orc.intt(len(a1), limb) == v)
            a1.append(limb)
            a2.append(orc.ntt(len(a2), np.eye(1, orc.N, 0, dtype=np.uint64)[0]))
    assert len(a1) == level
    b1 = np.stack([rng.integers(0, q, orc.N, dtype=np.uint64) for q in orc.q[:level]])
    b2 = np.stack([rng.integers(0, q, orc.N, dtype=np.uint64) for q in orc.q[:level]])
    ct1, ct2 = np.stack([b1, np.stack(a1)]), np.stack([b2, np.stack(a2)])
    evk = random_evk(orc, 3)
    want_relin, want_out = orc.he_mul(level, ct1, ct2, evk)
    relin, out = lib.he_mul(level, lib.to_device(ct1), lib.to_device(ct2), lib.to_device(evk))
    assert np.array_equal(lib.to_host(relin), want_relin)
    assert np.array_equal(lib.to_host(out), want_out)


def test_he_mul_deterministic_repeats():
    lib, orc = contexts("n16_L24")
    level = 24
    ct1 = lib.to_device(synth.random_ciphertext(7, orc.q[:level], orc.N))
    ct2 = lib.to_device(synth.random_ciphertext(8, orc.q[:level], orc.N))
    evk = lib.to_device(random_evk(orc, 3))
    _, first = lib.he_mul(level, ct1, ct2, evk, relin=False)
    ref = lib.to_host(first).copy()
    for _ in range(20):
        _, o = lib.he_mul(level, ct1, ct2, evk, relin=False)
        assert np.array_equal(lib.to_host(o), ref)


def test_errors_are_reported():
    P = need_gpu()
    lib, orc = contexts("n12_L3")
    ct = lib.to_device(synth.random_ciphertext(1, orc.q, orc.N))
    evk = lib.to_device(random_evk(orc))
    with pytest.raises(P.HeError, match="level"):
        lib.he_mul(0, ct, ct, evk)
    with pytest.raises(P.HeError, match="level"):
        lib.he_mul(4, ct, ct, evk)
    with pytest.raises(P.HeError, match="alias"):
        lib.he_mul(3, ct, ct, evk, out_relin=ct, rescale=False)
    small_ws = lib.empty(16)
    with pytest.raises(P.HeError, match="workspace"):
        lib.he_mul(3, ct, ct, evk, ws=small_ws)
