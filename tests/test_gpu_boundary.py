"""GPU: the boundary's ownership and metadata calls -- context tables in
caller memory or library memory (identical results), ciphertext import and
export with level and scale, he_mul_ct / he_rescale_ct scale bookkeeping
(Sec. III-A), and the argument errors they report."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_common import contexts, log, need_gpu, random_evk

pytestmark = pytest.mark.gpu


def test_ct_import_export_and_scale_metadata():
    P = need_gpu()
    lib, orc = contexts("n16_L24")
    level = 9
    a_h = synth.random_ciphertext(31, orc.q[:level], orc.N)
    b_h = synth.random_ciphertext(32, orc.q[:level], orc.N)
    evk_h = random_evk(orc, 33)
    evk = lib.to_device(evk_h)
    a = lib.ct_import(a_h, level, 2.0 ** 40)
    b = lib.ct_import(b_h, level, 2.0 ** 41)
    assert (a.level, a.scale) == (level, 2.0 ** 40)
    assert np.array_equal(lib.ct_export(a), a_h)
    relin, out = lib.mul_ct(a, b, evk)
    want_relin, want_out = orc.he_mul(level, a_h, b_h, evk_h)
    assert np.array_equal(lib.ct_export(relin), want_relin)
    assert np.array_equal(lib.ct_export(out), want_out)
    assert relin.level == level and relin.scale == 2.0 ** 81
    assert out.level == level - 1 and out.scale == 2.0 ** 81 / orc.q[level - 1]
    r2 = lib.rescale_ct(relin)
    assert r2.level == level - 1 and r2.scale == out.scale
    assert np.array_equal(lib.ct_export(r2), want_out)
    log("ct descriptors ok")


def test_ct_errors():
    P = need_gpu()
    lib, orc = contexts("n12_L3")
    h = synth.random_ciphertext(1, orc.q, orc.N)
    bad = h.copy()
    bad[1, 2, 7] = orc.q[2]          # not below q_2
    with pytest.raises(P.HeError, match="below"):
        lib.ct_import(bad, 3, 2.0 ** 40)
    with pytest.raises(P.HeError, match="scale"):
        lib.ct_import(h, 3, -1.0)
    a = lib.ct_import(h, 3, 2.0 ** 40)
    b = lib.ct_import(h[:, :2], 2, 2.0 ** 40)
    evk = lib.to_device(random_evk(orc))
    with pytest.raises(P.HeError, match="level"):
        lib.mul_ct(a, b, evk)
    ct = lib.to_device(h)
    with pytest.raises(P.HeError, match="overlap"):
        lib.rescale(3, ct, out=ct)     # in place: rejected, not silently wrong
    shifted = ct.view(-1)[orc.N: 5 * orc.N].view(2, 2, orc.N)   # output one limb past the input's start
    with pytest.raises(P.HeError, match="overlap"):
        lib.rescale(3, ct, out=shifted)


def test_library_owned_and_caller_owned_tables_agree():
    """A context whose tables the library allocates (d_tables = NULL) and
    the binding's context (tables in torch memory) give the same HE Mul;
    too little table memory is HE_ENOMEM."""
    import torch
    P = need_gpu()
    L = P.load_library()
    lib, orc = contexts("n12_L3")
    q = (ctypes.c_uint64 * orc.L)(*orc.q)
    p = (ctypes.c_uint64 * orc.K)(*orc.p)
    h = ctypes.c_void_p()
    small = torch.empty(16, dtype=torch.int64, device="cuda")
    assert L.he_ctx_create(orc.log_n, orc.L, orc.K, orc.dnum, q, p, 0, ctypes.c_void_p(small.data_ptr()), 128,
                           ctypes.byref(h)) == -3
    assert L.he_ctx_create(orc.log_n, orc.L, orc.K, orc.dnum, q, p, 0, None, 0, ctypes.byref(h)) == 0
    try:
        assert L.he_ctx_table_bytes(h) == lib.table_bytes()
        ct1 = lib.to_device(synth.random_ciphertext(3, orc.q, orc.N))
        ct2 = lib.to_device(synth.random_ciphertext(4, orc.q, orc.N))
        evk = lib.to_device(random_evk(orc, 5))
        ws = lib.workspace(3)
        out = lib.empty(2, 2, orc.N)
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        assert L.he_mul(h, 3, ctypes.c_void_p(ct1.data_ptr()), ctypes.c_void_p(ct2.data_ptr()),
                        ctypes.c_void_p(evk.data_ptr()), None, ctypes.c_void_p(out.data_ptr()),
                        ctypes.c_void_p(ws.data_ptr()), ws.numel() * 8, st) == 0
        _, want = lib.he_mul(3, ct1, ct2, evk, relin=False)
        torch.cuda.synchronize()
        assert np.array_equal(lib.to_host(out), lib.to_host(want))
    finally:
        L.he_ctx_destroy(h)
