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
    for fused in (0, 1, 2, 3):  # none, every pair, the pairs of >= 2 or 3 digits
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


@pytest.mark.parametrize("sched", [(4096, 2048, 1, 0, 8), (2048, 2048, 2, 0, 8), (4096, 1024, 4, 1, 8),
                                   (2048, 1024, 3, 1, 8), (4096, 2048, 8, 0, 8), (4096, 1024, 1, 1, 8),
                                   (2048, 1024, 2, 1, 8), (4096, 1024, 2, 0, 8), (2048, 1024, 1, 0, 16),
                                   (4096, 2048, 2, 0, 16), (2048, 2048, 1, 1, 16), (4096, 1024, 3, 0, 16),
                                   (2048, 1024, 1, 2, 8), (4096, 1024, 2, 3, 16)])
def test_batch_schedules_match_oracle(sched):
    """Every tile choice, NTT radix, chunk split and the fused inner-product
    pass (for every pair, or only for the pairs of at least 2 or 3 digits,
    the others taking the separate launches in the same batch) give the
    oracle's results for every pair, eagerly and on repeated graph
    replays."""
    lib, orc, evk, items, want = _setup("n16_L24", N16_LEVELS, 500, 7, 3)
    log("batch sched", sched, N16_LEVELS)
    bt = lib.batch(items)
    bt.set_sched(*sched)
    assert bt.sched() == {"cols_tile": sched[0], "blocks_tile": sched[1], "chunks": sched[2], "ip_fused": sched[3],
                          "radix": sched[4]}
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
    assert sc["ip_fused"] in (0, 1, 2, 3) and sc["radix"] in (8, 16)
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
        bt.set_sched(4096, 2048, 1, 5)  # ip_fused: a digit threshold 0..4
    with pytest.raises(P.HeError, match="radix"):
        bt.set_sched(4096, 2048, 1, 0, 16)  # radix 16 only at N = 2^16
    with pytest.raises(P.HeError, match="radix"):
        bt.set_sched(4096, 2048, 1, 0, 32)
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


def test_batch_group_mixed_rings_match_oracle():
    """Batches of three ring sizes (N = 2^12, 2^15, 2^16) run as one group,
    each ring on its own stream, captured into one HIP graph: every pair of
    every ring gives the oracle's results, eagerly and on repeated replays
    with other work in between; later schedule changes are refused."""
    import torch

    import paper_2003_04510_amd as P
    rings = [("n12_L3", (3, 2, 3), 910), ("n15_L12", (12, 4, 9, 2), 920), ("n16_L24", (24, 7, 15), 930)]
    setups = []
    for wname, levels, seed in rings:
        lib, orc, evk, items, want = _setup(wname, levels, seed, 12, 2)
        setups.append((wname, lib, evk, items, want, lib.batch(items)))
    log("batch group", [r[0] for r in rings])
    grp = P.BatchGroup([s[5] for s in setups])
    evks = [s[2] for s in setups]
    for k, use_graph in enumerate((False, True, True, True)):
        for _, _, _, items, _, _ in setups:
            _clear(items)
        torch.cuda.synchronize()
        grp.run(evks, use_graph=use_graph)
        if k == 2:
            torch.cuda.synchronize()
            scratch = torch.ones(1 << 20, device="cuda").sum()   # other work between replays
            assert float(scratch) == float(1 << 20)
        torch.cuda.synchronize()
        for wname, lib, _, items, want, _ in setups:
            _check_all(lib, items, want, ("group", wname, k))
    # a schedule change after grouping is refused before any launch, and
    # chunked batches do not form groups (a group recapture after one batch
    # switched to a chunked schedule crashed the host process once; those
    # two paths are off, see the design notes)
    n16 = setups[2][5]
    n16.set_sched(4096, 2048, 2, 1)
    with pytest.raises(P.HeError, match="schedule"):
        grp.run(evks, use_graph=True)
    grp.close()
    with pytest.raises(P.HeError, match="chunk"):
        P.BatchGroup([s[5] for s in setups])
    for s in setups:
        s[5].close()
