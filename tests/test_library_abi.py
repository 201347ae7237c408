"""CPU-side checks of the C ABI: the built library loads and exports every
function include/he_mi355x.h declares; host-side logic (prime search) agrees
with the oracle.  No device work."""
import ctypes
import os
import re

import numpy as np

import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "he_mi355x.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(he_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("he_ctx_create", "he_keygen", "he_encrypt", "he_decrypt", "he_mul", "he_rescale"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2003_04510_amd as P
    lib = P.load_library()
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_library_prime_search_matches_oracle():
    import paper_2003_04510_amd as P
    for w in synth.WORKLOADS.values():
        assert P.workload_primes(w) == oracle.workload_primes(w), w.name


def test_library_primality_against_a_sieve():
    """The library's prime search (its own Baillie-PSW test, written apart
    from the oracle's Miller-Rabin) lists exactly the primes = 1 mod 4 below
    2^21 that a sieve finds, strong base-2 pseudoprimes such as 15841,
    29341, 1373653 among the candidates it must reject."""
    import numpy as np

    import paper_2003_04510_amd as P
    n = 1 << 21
    sieve = np.ones(n, dtype=bool)
    sieve[:2] = False
    for i in range(2, int(n ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = False
    want = [int(x) for x in np.nonzero(sieve)[0][::-1] if x % 4 == 1 and x > 4]
    got = P.binding.gen_primes(1, 21, len(want))
    assert got == want
    for psp in (15841, 29341, 1373653):
        assert pow(2, psp - 1, psp) == 1 and not sieve[psp] and psp % 4 == 1


def test_status_strings_and_argument_errors():
    import paper_2003_04510_amd as P
    lib = P.load_library()
    assert lib.he_status_str(0) == b"ok"
    assert lib.he_status_str(-6) == b"busy"
    h = ctypes.c_void_p()
    # null moduli -> HE_EINVAL before any device call
    assert lib.he_ctx_create(16, 3, 1, 3, None, None, 0, None, 0, ctypes.byref(h)) == -1
    q = (ctypes.c_uint64 * 3)(*oracle.workload_primes(synth.CFG_N12)[0])
    p = (ctypes.c_uint64 * 1)(*oracle.workload_primes(synth.CFG_N12)[1])
    assert lib.he_ctx_create(11, 3, 1, 3, q, p, 0, None, 0, ctypes.byref(h)) == -5   # log_n out of range
    assert lib.he_ctx_create(12, 3, 1, 9, q, p, 0, None, 0, ctypes.byref(h)) == -1   # dnum > L
    bad = (ctypes.c_uint64 * 3)(q[0], q[1], q[1])
    assert lib.he_ctx_create(12, 3, 1, 3, bad, p, 0, None, 0, ctypes.byref(h)) == -1  # duplicate
    with pytest.raises(Exception):
        P.binding.gen_primes(12, 70, 1)


def _table_bytes(w):
    import paper_2003_04510_amd as P
    lib = P.load_library()
    lib.he_ctx_device_bytes.restype = ctypes.c_size_t
    q, p = oracle.workload_primes(w)
    qa = (ctypes.c_uint64 * len(q))(*q)
    pa = (ctypes.c_uint64 * len(p))(*p)
    return lib.he_ctx_device_bytes(w.log_n, len(q), len(p), w.dnum, qa, pa), qa, pa


def test_context_table_size_query():
    """he_ctx_device_bytes sizes the caller-owned table memory without a
    device: twice N 16-byte twiddle entries per modulus (forward and
    inverse) plus the per-level conversion constants; 0 for invalid
    parameters."""
    for w in (synth.CFG_N12, synth.CFG_N16, synth.CFG_N17):
        n, _, _ = _table_bytes(w)
        tw = 2 * (w.L + w.K) * w.N * 16
        assert tw < n < tw + (64 << 20), (w.name, n)
    import paper_2003_04510_amd as P
    lib = P.load_library()
    n, q, p = _table_bytes(synth.CFG_N12)
    assert lib.he_ctx_device_bytes(11, 3, 1, 3, q, p) == 0
    assert lib.he_ctx_device_bytes(12, 3, 1, 4, q, p) == 0
    assert lib.he_ctx_device_bytes(12, 3, 1, 3, None, p) == 0


def test_server_arena_and_budget_errors_without_device():
    import paper_2003_04510_amd as P
    lib = P.load_library()
    cfg = P.binding.ServerCfg(1 << 30, 8, 2, 4, 100)
    lib.he_server_arena_min_bytes.restype = ctypes.c_size_t
    n = lib.he_server_arena_min_bytes(ctypes.byref(cfg))
    assert n > 0 and n % 256 == 0
    assert lib.he_server_arena_min_bytes(ctypes.byref(P.binding.ServerCfg(1 << 30, 0, 2, 0, 0))) == 0
    h = ctypes.c_void_p()
    assert lib.he_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
    rid = ctypes.c_uint32()
    assert lib.he_server_add_ring(h, None, None, None, 0, ctypes.byref(rid)) == -1
    assert lib.he_server_submit(h, 0, 1, 3, None, None, None) == -1
    lib.he_server_destroy(h)


class _FakeCtx:
    """Just the fields the binding's argument checks read."""


def test_binding_rejects_bad_tensors_before_any_call():
    """The binding checks device, dtype, contiguity and size of every tensor
    it hands to the library, and the length of host draws, before any C
    call (CPU tensors stand in for device ones here)."""
    import torch

    import paper_2003_04510_amd as P
    ctx = P.Context.__new__(P.Context)
    ctx.torch, ctx.N, ctx.L, ctx.device, ctx.wdtype = torch, 16, 3, 0, torch.int64
    t = torch.zeros(2 * 3 * 16, dtype=torch.int64)
    with pytest.raises(P.HeError, match="cuda"):
        ctx._ct(t, 3, "x")
    with pytest.raises(P.HeError, match="level"):
        ctx._ct(t, 4, "x")
    with pytest.raises(P.HeError, match="missing"):
        ctx._dev(None, 1, "x")
    with pytest.raises(P.HeError, match="elements"):
        P.binding._host(np.zeros(15), 16, np.int64, "s")
    assert P.binding._host(np.zeros(16), 16, np.int64, "s").dtype == np.int64


def test_big_context_argument_errors():
    """The non-RNS path rejects unsupported parameters before any device call."""
    import paper_2003_04510_amd as P
    lib = P.load_library()
    h = ctypes.c_void_p()
    assert lib.he_big_ctx_create(16, 1200, 0, None) == -1        # null out
    assert lib.he_big_ctx_create(11, 1200, 0, ctypes.byref(h)) == -5  # log_n below 12
    assert lib.he_big_ctx_create(16, 1217, 0, ctypes.byref(h)) == -5  # log Q above 1216
    assert lib.he_big_ctx_create(16, 63, 0, ctypes.byref(h)) == -5    # log Q below 64
    assert lib.he_big_ct_bytes(None) == 0 and lib.he_big_workspace_bytes(None) == 0
    assert lib.he_big_mul(None, 10, None, None, None, None, 0, None, 0, None) == -1
