"""GPU: a batched HE Mul (pairs of uneven levels in one sequence of batched
stage kernels, optionally replayed from a HIP graph) gives, pair by pair and
under every schedule, exactly the oracle's relinearized and rescaled
ciphertexts."""
import functools

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


@functools.lru_cache(maxsize=None)
def _expected(wname, levels, seed, evk_seed):
    """Host operands, evk and the oracle's (relin, out) for every pair."""
    _, orc = contexts(wname)
    evk = random_evk(orc, evk_seed)
    pairs = _pairs(orc, levels, seed)
    want = [orc.he_mul(lv, a, b, evk) for lv, a, b in pairs]
    return pairs, evk, want


def _check_all(lib, items, want, tag):
    """Every pair's outputs against the oracle, element by element."""
    for i, ((_, _, _, relin, out), (w_relin, w_out)) in enumerate(zip(items, want)):
        assert np.array_equal(lib.to_host(out), w_out), (tag, i, "out")
        if relin is not None:
            assert np.array_equal(lib.to_host(relin), w_relin), (tag, i, "relin")


def _clear(items):
    for _, _, _, relin, out in items:
        out.fill_(0)
        if relin is not None:
            relin.fill_(0)


def _setup(wname, levels, seed, evk_seed, relin_every):
    lib, orc = contexts(wname)
    pairs, evk_h, want = _expected(wname, tuple(levels), seed, evk_seed)
    evk = lib.to_device(evk_h)
    dev = [(lv, lib.to_device(a), lib.to_device(b)) for lv, a, b in pairs]
    items = [(lv, a, b, lib.empty(2, lv, orc.N) if i % relin_every == 0 else None, lib.empty(2, lv - 1, orc.N))
             for i, (lv, a, b) in enumerate(dev)]
    return lib, orc, evk, items, want


def _run_check(lib, bt, items, evk, want, use_graph, tag):
    import torch
    _clear(items)
    torch.cuda.synchronize()
    bt.run(evk, use_graph=use_graph)
    torch.cuda.synchronize()
    _check_all(lib, items, want, tag)


@pytest.mark.parametrize("wname,levels", [
    ("n12_L3", [3, 2, 3, 2, 3]),
    ("n16_L24", [24, 4, 17, 9, 24, 5]),
])
def test_batch_matches_oracle(wname, levels):
    lib, orc, evk, items, want = _setup(wname, levels, 300, 5, 2)
    log("batch", wname, levels)
    bt = lib.batch(items)
    for k, use_graph in enumerate((False, True, True)):
        _run_check(lib, bt, items, evk, want, use_graph, (wname, k))
    bt.close()


def test_batch_n12_all_levels_every_schedule():
    """N = 2^12: every level, each schedule that exists at this ring
    (default tiles; fused pass or not; 1..4 chunks), all pairs."""
    levels = [3, 1, 2, 3, 2, 1, 3, 3]
    lib, orc, evk, items, want = _setup("n12_L3", levels, 350, 4, 1)
    # level 1 has no rescaled output: its out buffer is unused by he_mul, so
    # give those pairs the relinearized output only
    items = [(lv, a, b, relin, out if lv >= 2 else None) for lv, a, b, relin, out in items]
    log("batch n12 every schedule", levels)
    bt = lib.batch(items)
    sc = bt.sched()
    import torch
    for fused in (0, 1):
        for chunks in (1, 2, 4):
            bt.set_sched(sc["cols_tile"], sc["blocks_tile"], chunks, fused)
            for k, use_graph in enumerate((False, True, True)):
                for _, _, _, relin, out in items:
                    relin.fill_(0)
                    if out is not None:
                        out.fill_(0)
                torch.cuda.synchronize()
                bt.run(evk, use_graph=use_graph)
                torch.cuda.synchronize()
                for i, ((lv, _, _, relin, out), (w_relin, w_out)) in enumerate(zip(items, want)):
                    assert np.array_equal(lib.to_host(relin), w_relin), (fused, chunks, k, i)
                    if out is not None:
                        assert np.array_equal(lib.to_host(out), w_out), (fused, chunks, k, i)
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


N16_LEVELS = (24, 4, 17, 9, 24, 5, 12, 20)


@pytest.mark.parametrize("sched", [(4096, 2048, 1, 0), (2048, 2048, 2, 0), (4096, 1024, 4, 1), (2048, 1024, 3, 1),
                                   (4096, 2048, 8, 0), (4096, 1024, 1, 1), (2048, 1024, 2, 1), (4096, 1024, 2, 0)])
def test_batch_schedules_match_oracle(sched):
    """Every tile choice, chunk split and the fused inner-product pass give
    the oracle's results for every pair, eagerly and on repeated graph
    replays."""
    lib, orc, evk, items, want = _setup("n16_L24", N16_LEVELS, 500, 7, 3)
    log("batch sched", sched, N16_LEVELS)
    bt = lib.batch(items)
    bt.set_sched(*sched)
    assert bt.sched() == {"cols_tile": sched[0], "blocks_tile": sched[1], "chunks": sched[2], "ip_fused": sched[3]}
    for k, use_graph in enumerate((False, True, True, True)):
        _run_check(lib, bt, items, evk, want, use_graph, (sched, k))
    bt.close()


def test_batch_autotune_keeps_results():
    levels = (24, 6, 15, 24, 9, 3)
    lib, orc, evk, items, want = _setup("n16_L24", levels, 600, 7, 3)
    log("batch autotune", levels)
    bt = lib.batch(items)
    sc, ms = bt.autotune(evk, reps=1)
    log("tuned", sc, ms)
    assert ms > 0
    assert sc == bt.sched()
    assert sc["cols_tile"] in (2048, 4096) and sc["blocks_tile"] in (1024, 2048) and sc["chunks"] in (1, 2, 4)
    assert sc["ip_fused"] in (0, 1)
    for k, use_graph in enumerate((True, False, True)):
        _run_check(lib, bt, items, evk, want, use_graph, ("tuned", k))
    bt.close()


def test_batch_sched_errors():
    import paper_2003_04510_amd as P
    lib, orc, evk, items, want = _setup("n12_L3", (3, 2), 700, 8, 10 ** 9)
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
    _check_all(lib, items, want, "errors")
    bt.close()


@pytest.mark.parametrize("wname,levels", [("n17_L45", (45, 17, 3)), ("n15_L12", (12, 5, 9, 2))])
def test_fused_ip_other_rings(wname, levels):
    """The fused mod-up blocks + inner-product pass at N = 2^17 (512-point
    blocks, radix 2^5) and N = 2^15 gives the oracle's results."""
    lib, orc, evk, items, want = _setup(wname, levels, 800, 9, 10 ** 9)
    items[0] = (items[0][0], items[0][1], items[0][2], lib.empty(2, levels[0], orc.N), items[0][4])
    log("fused ip", wname, levels)
    bt = lib.batch(items)
    sc = bt.sched()
    bt.set_sched(sc["cols_tile"], sc["blocks_tile"], 1, 1)
    for k, use_graph in enumerate((False, True, True)):
        _run_check(lib, bt, items, evk, want, use_graph, (wname, k))
    bt.close()


@pytest.mark.parametrize("wname,levels", [("n16_L24_d24", (24, 7, 16)), ("n16_L24_d1", (24, 3, 11))])
def test_batch_dnum_variants(wname, levels):
    """Batches with 24 digits (no fused pass: the tuner skips it, set_sched
    refuses it) and with one 24-prime digit give the oracle's results."""
    import paper_2003_04510_amd as P
    lib, orc, evk, items, want = _setup(wname, levels, 800, 9, 10 ** 9)
    items[0] = (items[0][0], items[0][1], items[0][2], lib.empty(2, levels[0], orc.N), items[0][4])
    log("batch dnum variant", wname, levels)
    bt = lib.batch(items)
    if orc.dnum > 4:
        with pytest.raises(P.HeError):
            bt.set_sched(4096, 1024, 1, 1)
    sc, _ = bt.autotune(evk, reps=1)
    if orc.dnum > 4:
        assert sc["ip_fused"] == 0
    for k, use_graph in enumerate((True, True)):
        _run_check(lib, bt, items, evk, want, use_graph, (wname, k))
    bt.close()
