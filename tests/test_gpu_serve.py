"""GPU: the continuous-batching server.  Requests of three ring sizes and
random levels arrive in bursts while earlier batches are still running;
every result equals the oracle's HE Mul of the same operands, bit for bit,
and also the same HE Mul computed alone (plain he_mul); the server's
bookkeeping (admission by footprint under a small budget, bounded queue,
coalescing hold, ids, latencies) is consistent."""
import functools
import time

import numpy as np
import pytest

import synth
from gpu_common import contexts, log, random_evk

pytestmark = pytest.mark.gpu

RINGS = ("n12_L3", "n15_L12", "n16_L24")


@functools.lru_cache(maxsize=None)
def _host_ring(wname):
    _, orc = contexts(wname)
    evk = random_evk(orc, 21)
    ops = [synth.random_ciphertext(50 + k, orc.q, orc.N) for k in range(3)]
    return evk, ops


@functools.lru_cache(maxsize=None)
def _oracle(wname, ia, ib, lv):
    _, orc = contexts(wname)
    evk, ops = _host_ring(wname)
    return orc.he_mul(lv, ops[ia][:, :lv], ops[ib][:, :lv], evk)[1]


def _serve(hold_us, nreq, seed):
    import torch

    import paper_2003_04510_amd as P
    rng = np.random.default_rng(seed)
    rings = []
    for wname in RINGS:
        lib, orc = contexts(wname)
        evk_h, ops_h = _host_ring(wname)
        rings.append((wname, lib, orc, lib.to_device(evk_h), [lib.to_device(o) for o in ops_h]))
    srv = P.Server(hbm_budget=3 << 30, max_batch=8, max_inflight=2, hold_us=hold_us)
    # arenas deliberately small so that admission by footprint binds
    arena = {12: 64 << 20, 15: 400 << 20, 16: 800 << 20}
    rid = [srv.add_ring(lib, evk, arena[lib.log_n]) for _, lib, _, evk, _ in rings]
    reqs = {}
    for i in range(nreq):
        r = int(rng.choice(3, p=[0.3, 0.4, 0.3]))
        wname, lib, orc, evk, ops = rings[r]
        lv = int(rng.integers(2, orc.L + 1))
        ia, ib = int(rng.integers(0, 3)), int(rng.integers(0, 3))
        a = ops[ia][:, :lv, :].contiguous()
        b = ops[ib][:, :lv, :].contiguous()
        out = lib.empty(2, lv - 1, orc.N)
        reqs[i] = (r, lv, ia, ib, a, b, out)
        torch.cuda.synchronize()  # the server's streams do not wait for torch's
        srv.submit(rid[r], i, lv, a, b, out)
        if i % 7 == 0:
            srv.progress()
    log("submitted", nreq, srv.stats())
    done = {}
    t0 = time.time()
    while len(done) < nreq and time.time() - t0 < 60:
        srv.progress()
        for k, lat in srv.poll():
            assert k not in done and lat > 0
            done[k] = lat
    st = srv.stats()
    log("server", st)
    assert len(done) == nreq and st["completed"] == nreq and st["queued"] == 0 and st["inflight"] == 0
    assert st["batches"] < nreq  # requests were batched
    for i, (r, lv, ia, ib, a, b, out) in reqs.items():
        wname, lib, orc, evk, ops = rings[r]
        got = lib.to_host(out)
        assert np.array_equal(got, _oracle(wname, ia, ib, lv)), (i, wname, lv)
        _, alone = lib.he_mul(lv, a, b, evk, relin=False)
        assert np.array_equal(got, lib.to_host(alone)), (i, wname, lv)
    srv.close()
    return st


def test_served_results_match_oracle_and_alone():
    _serve(hold_us=0, nreq=48, seed=9)


def test_served_with_coalescing_hold():
    st = _serve(hold_us=2000, nreq=40, seed=10)
    assert st["batches"] <= 30


def test_server_rejects_oversized_bad_levels_and_full_queue():
    import paper_2003_04510_amd as P
    lib, orc = contexts("n12_L3")
    evk = lib.to_device(random_evk(orc, 3))
    fixed = lib.table_bytes() + lib.evk_bytes()
    srv = P.Server(hbm_budget=fixed + (1 << 20), max_batch=4, max_inflight=1, max_queue=2)
    with pytest.raises(P.HeError, match="budget"):
        srv.add_ring(lib, evk, 2 << 20)  # tables + evk + arena over the budget
    r = srv.add_ring(lib, evk, 1 << 20)  # too small for any request at N=2^12
    a = lib.to_device(synth.random_ciphertext(1, orc.q, orc.N))
    out = lib.empty(2, 2, orc.N)
    with pytest.raises(P.HeError):
        srv.submit(r, 0, 3, a, a, out)
    with pytest.raises(P.HeError):
        srv.submit(r, 1, 1, a, a, out)
    srv.close()
    # bounded queue: the third request of a ring that launches nothing yet
    srv = P.Server(hbm_budget=1 << 30, max_batch=4, max_inflight=1, max_queue=2)
    r = srv.add_ring(lib, evk, 64 << 20)
    outs = [lib.empty(2, 2, orc.N) for _ in range(3)]
    srv.submit(r, 10, 3, a, a, outs[0])
    srv.submit(r, 11, 3, a, a, outs[1])
    with pytest.raises(P.HeBusy):
        srv.submit(r, 12, 3, a, a, outs[2])
    done = set()
    t0 = time.time()
    while len(done) < 2 and time.time() - t0 < 30:
        srv.progress()
        done |= {k for k, _ in srv.poll()}
    assert done == {10, 11}
    srv.submit(r, 12, 3, a, a, outs[2])   # room again
    while 12 not in done and time.time() - t0 < 30:
        srv.progress()
        done |= {k for k, _ in srv.poll()}
    assert 12 in done
    _, want = orc.he_mul(3, synth.random_ciphertext(1, orc.q, orc.N), synth.random_ciphertext(1, orc.q, orc.N),
                         random_evk(orc, 3))
    for o in outs:
        assert np.array_equal(lib.to_host(o), want)
    srv.close()
