"""GPU: the 32-bit-word variant (the paper's GPU word size, Table VI: primes
below 2^30, residues in 32-bit words).  he_mul32 on a 32-bit-word context
gives, widened, exactly the oracle's relinearized and rescaled ciphertexts,
and exactly what he_mul gives on 64-bit words for the same primes."""
import functools

import numpy as np
import pytest

import synth
from gpu_common import contexts, log, need_gpu, random_evk

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def ctx32(wname):
    P = need_gpu()
    w = synth.WORKLOADS[wname]
    lib = P.Context.for_workload(w, word32=True)
    assert lib.word32 and lib.ct_bytes(1) == 2 * w.N * 4
    return lib


@pytest.mark.parametrize("wname,level", [("n12_L6_w30", 6), ("n12_L6_w30", 4), ("n12_L6_w30", 2),
                                         ("n16_L40_w30", 40), ("n16_L40_w30", 11), ("n16_L40_w30", 2)])
def test_he_mul32_matches_oracle_and_64bit_words(wname, level):
    lib64, orc = contexts(wname)
    lib = ctx32(wname)
    assert lib.q == orc.q and lib.p == orc.p
    log("he_mul32", wname, level)
    ct1 = synth.random_ciphertext(70 + level, orc.q[:level], orc.N)
    ct2 = synth.random_ciphertext(90 + level, orc.q[:level], orc.N)
    evk = random_evk(orc, 11)
    relin, out = lib.he_mul(level, lib.to_device(ct1), lib.to_device(ct2), lib.to_device(evk))
    assert relin.dtype == lib.torch.int32
    want_relin, want_out = orc.he_mul(level, ct1, ct2, evk)
    assert np.array_equal(lib.to_host(relin), want_relin)
    if level >= 2:
        assert np.array_equal(lib.to_host(out), want_out)
    r64, o64 = lib64.he_mul(level, lib64.to_device(ct1), lib64.to_device(ct2), lib64.to_device(evk))
    assert np.array_equal(lib64.to_host(r64), lib.to_host(relin))
    assert np.array_equal(lib64.to_host(o64), lib.to_host(out))


def test_he_mul32_extreme_inputs():
    _, orc = contexts("n12_L6_w30")
    lib = ctx32("n12_L6_w30")
    level = 6
    ct = np.stack([np.stack([np.full(orc.N, q - 1, dtype=np.uint64) for q in orc.q[:level]])] * 2)
    evk = np.stack([np.stack([np.stack([np.full(orc.N, m - 1, dtype=np.uint64) for m in orc.moduli])] * 2)]
                   * orc.dnum)
    want_relin, want_out = orc.he_mul(level, ct, ct, evk)
    relin, out = lib.he_mul(level, lib.to_device(ct), lib.to_device(ct), lib.to_device(evk))
    assert np.array_equal(lib.to_host(relin), want_relin)
    assert np.array_equal(lib.to_host(out), want_out)


def test_word_size_errors():
    P = need_gpu()
    lib64, orc = contexts("n12_L6_w30")
    lib = ctx32("n12_L6_w30")
    L = P.load_library()
    assert L.he_ctx_word_bytes(lib._h) == 4 and L.he_ctx_word_bytes(lib64._h) == 8
    ct = synth.random_ciphertext(1, orc.q, orc.N)
    evk = random_evk(orc, 2)
    # he_mul on 32-bit words and he_mul32 on 64-bit words are refused
    a32, e32 = lib.to_device(ct), lib.to_device(evk)
    ws = lib.workspace(6)
    o = lib.empty(2, 5, orc.N)
    import ctypes
    st = ctypes.c_void_p(lib.torch.cuda.current_stream().cuda_stream)
    vp = ctypes.c_void_p
    assert L.he_mul(lib._h, 6, vp(a32.data_ptr()), vp(a32.data_ptr()), vp(e32.data_ptr()), None, vp(o.data_ptr()),
                    vp(ws.data_ptr()), ws.numel() * 8, st) == -5
    a64 = lib64.to_device(ct)
    assert L.he_mul32(lib64._h, 6, vp(a64.data_ptr()), vp(a64.data_ptr()), vp(a64.data_ptr()), None,
                      vp(o.data_ptr()), vp(ws.data_ptr()), ws.numel() * 8, st) == -5
    with pytest.raises(P.HeError, match="32-bit"):
        lib.to_device(np.array([1 << 32], dtype=np.uint64))
    with pytest.raises(P.HeError, match="dtype"):
        lib.he_mul(6, a64, a64, lib.to_device(evk))   # int64 tensors into a 32-bit-word context
    with pytest.raises(P.HeError):
        P.Context.for_workload(synth.CFG_N12, word32=True)   # 50-bit primes do not fit 32-bit words
