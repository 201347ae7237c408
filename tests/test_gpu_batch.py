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


def _run_check(lib, bt, items, dev, evk, use_graph, tag):
    import torch
    for _, _, _, relin, out in items:
        out.fill_(0)
        if relin is not None:
            relin.fill_(0)
    torch.cuda.synchronize()
    bt.run(evk, use_graph=use_graph)
    torch.cuda.synchronize()
    for i, ((lv, a, b), (_, _, _, relin, out)) in enumerate(zip(dev, items)):
        p_relin, p_out = lib.he_mul(lv, a, b, evk)
        assert np.array_equal(lib.to_host(out), lib.to_host(p_out)), (tag, i)
        if relin is not None:
            assert np.array_equal(lib.to_host(relin), lib.to_host(p_relin)), (tag, i)


def _batch_n16(levels, seed):
    lib, orc = contexts("n16_L24")
    evk = lib.to_device(random_evk(orc, 7))
    dev = [(lv, lib.to_device(a), lib.to_device(b)) for lv, a, b in _pairs(orc, levels, seed)]
    items = [(lv, a, b, lib.empty(2, lv, orc.N) if i % 3 == 0 else None, lib.empty(2, lv - 1, orc.N))
             for i, (lv, a, b) in enumerate(dev)]
    return lib, evk, dev, items


@pytest.mark.parametrize("sched", [(4096, 2048, 1, 0), (2048, 2048, 2, 0), (4096, 1024, 4, 1), (2048, 1024, 3, 1),
                                   (4096, 2048, 8, 0), (4096, 1024, 1, 1)])
def test_batch_schedules_bit_exact(sched):
    """Every tile choice and chunk split gives the plain he_mul results,
    eagerly and on repeated graph replays."""
    levels = [24, 4, 17, 9, 24, 5, 12, 20]
    lib, evk, dev, items = _batch_n16(levels, 500)
    log("batch sched", sched, levels)
    bt = lib.batch(items)
    bt.set_sched(*sched)
    assert bt.sched() == {"cols_tile": sched[0], "blocks_tile": sched[1], "chunks": sched[2], "ip_fused": sched[3]}
    for k, use_graph in enumerate((False, True, True, True)):
        _run_check(lib, bt, items, dev, evk, use_graph, (sched, k))
    bt.close()


def test_batch_autotune_keeps_results():
    levels = [24, 6, 15, 24, 9, 3]
    lib, evk, dev, items = _batch_n16(levels, 600)
    log("batch autotune", levels)
    bt = lib.batch(items)
    sc, ms = bt.autotune(evk, reps=1)
    assert ms > 0
    assert sc == bt.sched()
    assert sc["cols_tile"] in (2048, 4096) and sc["blocks_tile"] in (1024, 2048) and sc["chunks"] in (1, 2, 4)
    assert sc["ip_fused"] in (0, 1)
    for k, use_graph in enumerate((True, False, True)):
        _run_check(lib, bt, items, dev, evk, use_graph, ("tuned", k))
    bt.close()


def test_batch_sched_errors():
    import paper_2003_04510_amd as P
    lib, orc = contexts("n12_L3")
    evk = lib.to_device(random_evk(orc, 8))
    dev = [(lv, lib.to_device(a), lib.to_device(b)) for lv, a, b in _pairs(orc, [3, 2], 700)]
    items = [(lv, a, b, None, lib.empty(2, lv - 1, orc.N)) for lv, a, b in dev]
    bt = lib.batch(items)
    with pytest.raises(P.HeError, match="EUNSUPPORTED|not available"):
        bt.set_sched(2048, 1024, 1)   # only the default tiles exist at N = 2^12
    with pytest.raises(P.HeError):
        bt.set_sched(4096, 2048, 0)
    with pytest.raises(P.HeError):
        bt.set_sched(4096, 2048, 3)   # more chunks than pairs
    with pytest.raises(P.HeError):
        bt.set_sched(4096, 2048, 1, 2)  # ip_fused is 0 or 1
    bt.set_sched(4096, 2048, 2, 1)   # the fused pass at N = 2^12
    for _ in range(2):
        bt.run(evk, use_graph=True)
    import torch
    torch.cuda.synchronize()
    for (lv, a, b), (_, _, _, _, out) in zip(dev, items):
        assert np.array_equal(lib.to_host(out), lib.to_host(lib.he_mul(lv, a, b, evk, relin=False)[1]))
    bt.close()


@pytest.mark.parametrize("wname,levels", [("n17_L45", [45, 17, 3]), ("n15_L12", [12, 5, 9, 2])])
def test_fused_ip_other_rings(wname, levels):
    """The fused mod-up blocks + inner-product pass at N = 2^17 (512-point
    blocks, radix 2^5) and N = 2^15 gives the plain he_mul results."""
    lib, orc = contexts(wname)
    evk = lib.to_device(random_evk(orc, 9))
    dev = [(lv, lib.to_device(a), lib.to_device(b)) for lv, a, b in _pairs(orc, levels, 800)]
    items = [(lv, a, b, lib.empty(2, lv, orc.N) if i == 0 else None, lib.empty(2, lv - 1, orc.N))
             for i, (lv, a, b) in enumerate(dev)]
    log("fused ip", wname, levels)
    bt = lib.batch(items)
    sc = bt.sched()
    bt.set_sched(sc["cols_tile"], sc["blocks_tile"], 1, 1)
    for k, use_graph in enumerate((False, True, True)):
        _run_check(lib, bt, items, dev, evk, use_graph, (wname, k))
    bt.close()


@pytest.mark.parametrize("wname,levels", [("n16_L24_d24", [24, 7, 16]), ("n16_L24_d1", [24, 3, 11])])
def test_batch_dnum_variants(wname, levels):
    """Batches with 24 digits (no fused pass: the tuner skips it, set_sched
    refuses it) and with one 24-prime digit give the plain he_mul results."""
    import paper_2003_04510_amd as P
    lib, orc = contexts(wname)
    log("batch dnum variant", wname, levels)
    evk = lib.to_device(random_evk(orc, 9))
    dev = [(lv, lib.to_device(a), lib.to_device(b)) for lv, a, b in _pairs(orc, levels, 800)]
    items = [(lv, a, b, lib.empty(2, lv, orc.N) if i == 0 else None, lib.empty(2, lv - 1, orc.N))
             for i, (lv, a, b) in enumerate(dev)]
    bt = lib.batch(items)
    if orc.dnum > 4:
        with pytest.raises(P.HeError):
            bt.set_sched(4096, 1024, 1, 1)
    sc, _ = bt.autotune(evk, reps=1)
    if orc.dnum > 4:
        assert sc["ip_fused"] == 0
    for k, use_graph in enumerate((True, True)):
        _run_check(lib, bt, items, dev, evk, use_graph, (wname, k))
    bt.close()
