"""GPU: a batched HE Mul (pairs of uneven levels in one sequence of batched
stage kernels, optionally replayed from a HIP graph) gives, pair by pair,
exactly the plain he_mul result, which is bit-exact to the oracle."""
import numpy as np
import pytest

import synth
from gpu_common import contexts, log, random_evk

pytestmark = pytest.mark.gpu


def _pairs(orc, levels, seed0):
    out = []
    for i, lv in enumerate(levels):
        out.append((lv, synth.random_ciphertext(seed0 + 2 * i, orc.q[:lv], orc.N),
                    synth.random_ciphertext(seed0 + 2 * i + 1, orc.q[:lv], orc.N)))
    return out


@pytest.mark.parametrize("wname,levels", [
    ("n12_L3", [3, 2, 3, 2, 3]),
    ("n16_L24", [24, 4, 17, 9, 24, 5]),
])
def test_batch_equals_plain_and_oracle(wname, levels):
    lib, orc = contexts(wname)
    log("batch", wname, levels)
    evk_h = random_evk(orc, 5)
    evk = lib.to_device(evk_h)
    pairs = _pairs(orc, levels, 300)
    dev = [(lv, lib.to_device(a), lib.to_device(b)) for lv, a, b in pairs]
    items = []
    for i, (lv, a, b) in enumerate(dev):
        relin = lib.empty(2, lv, orc.N) if i % 2 == 0 else None
        out = lib.empty(2, lv - 1, orc.N)
        items.append((lv, a, b, relin, out))
    bt = lib.batch(items)
    for use_graph in (False, True, True):
        for _, _, _, relin, out in items:
            out.fill_(0)
            if relin is not None:
                relin.fill_(0)
        bt.run(evk, use_graph=use_graph)
        for i, ((lv, a, b), (_, _, _, relin, out)) in enumerate(zip(dev, items)):
            p_relin, p_out = lib.he_mul(lv, a, b, evk)
            assert np.array_equal(lib.to_host(out), lib.to_host(p_out)), (i, use_graph)
            if relin is not None:
                assert np.array_equal(lib.to_host(relin), lib.to_host(p_relin)), (i, use_graph)
    # two pairs against the oracle directly
    for i in (0, len(pairs) - 1):
        lv, a, b = pairs[i]
        want_relin, want_out = orc.he_mul(lv, a, b, evk_h)
        assert np.array_equal(lib.to_host(items[i][4]), want_out)
    bt.close()


def test_batch_new_operands_between_runs():
    lib, orc = contexts("n12_L3")
    evk_h = random_evk(orc, 6)
    evk = lib.to_device(evk_h)
    a = lib.to_device(synth.random_ciphertext(1, orc.q, orc.N))
    b = lib.to_device(synth.random_ciphertext(2, orc.q, orc.N))
    out = lib.empty(2, 2, orc.N)
    bt = lib.batch([(3, a, b, None, out)])
    for seed in (10, 20):
        a_h = synth.random_ciphertext(seed, orc.q, orc.N)
        b_h = synth.random_ciphertext(seed + 1, orc.q, orc.N)
        a.copy_(lib.to_device(a_h))
        b.copy_(lib.to_device(b_h))
        bt.run(evk, use_graph=True)
        _, want = orc.he_mul(3, a_h, b_h, evk_h)
        assert np.array_equal(lib.to_host(out), want)
    bt.close()
