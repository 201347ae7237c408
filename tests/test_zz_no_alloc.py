"""GPU: he_mul_noalloc (the library's per-GPU scratch as workspace, no
allocation in the call) gives exactly he_mul's outputs, on two calls in a
row with the second on a smaller input, and rejects a level whose workspace
exceeds the scratch."""
import numpy as np
import pytest

import synth
from gpu_common import contexts, log, need_gpu, random_evk

pytestmark = pytest.mark.gpu


def _case(wname, level, seed):
    lib, orc = contexts(wname)
    a = lib.to_device(synth.random_ciphertext(seed, orc.q[:level], orc.N))
    b = lib.to_device(synth.random_ciphertext(seed + 1, orc.q[:level], orc.N))
    evk = lib.to_device(random_evk(orc, seed + 2))
    return lib, a, b, evk


def test_noalloc_matches_he_mul_twice_then_smaller():
    import torch
    P = need_gpu()
    cases = [("n15_L12", 12, 40), ("n12_L3", 2, 50)]   # the second call has the smaller input
    for wname, level, seed in cases:
        lib, a, b, evk = _case(wname, level, seed)
        log("noalloc", wname, level, lib.noalloc_bytes(level))
        assert lib.noalloc_bytes(level) <= 64 << 20
        relin = lib.empty(2, level, lib.N)
        out = lib.empty(2, level - 1, lib.N)
        relin.fill_(0)
        out.fill_(0)
        lib.he_mul_noalloc(level, a, b, evk, out_relin=relin, out=out)
        want_relin, want_out = lib.he_mul(level, a, b, evk)
        torch.cuda.synchronize()
        assert np.array_equal(lib.to_host(relin), lib.to_host(want_relin)), wname
        assert np.array_equal(lib.to_host(out), lib.to_host(want_out)), wname


def test_noalloc_rejects_oversized_and_bad_levels():
    P = need_gpu()
    lib, a, b, evk = _case("n16_L24", 24, 60)
    assert lib.noalloc_bytes(24) > 64 << 20
    out = lib.empty(2, 23, lib.N)
    with pytest.raises(P.HeError, match="scratch"):
        lib.he_mul_noalloc(24, a, b, evk, out=out)
    with pytest.raises(P.HeError, match="level"):
        lib.he_mul_noalloc(0, a, b, evk, out=out)
    # level 8 at N = 2^16 fits
    lv = 8
    a8, b8 = a[:, :lv].contiguous(), b[:, :lv].contiguous()
    o8 = lib.empty(2, lv - 1, lib.N)
    lib.he_mul_noalloc(lv, a8, b8, evk, out=o8)
    _, want = lib.he_mul(lv, a8, b8, evk, relin=False)
    assert np.array_equal(lib.to_host(o8), lib.to_host(want))
