"""GPU: the continuous-batching server.  Requests of two ring sizes and
random levels arrive in bursts while earlier batches are still running;
every result equals the same HE Mul computed alone (plain he_mul), bit for
bit, and the server's bookkeeping (admission under a small budget, ids,
latencies) is consistent."""
import time

import numpy as np
import pytest

import synth
from gpu_common import contexts, log, random_evk

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    import torch

    import paper_2003_04510_amd as P
    rng = np.random.default_rng(9)
    rings = []
    for wname in ("n12_L3", "n15_L12"):
        lib, orc = contexts(wname)
        evk = lib.to_device(random_evk(orc, 21))
        ops = [lib.to_device(synth.random_ciphertext(50 + k, orc.q, orc.N)) for k in range(4)]
        rings.append((lib, orc, evk, ops))
    # arenas deliberately small so that admission by footprint binds
    srv = P.Server(hbm_budget=1 << 30, max_batch=8, max_inflight=2)
    rid = [srv.add_ring(lib, evk, (64 << 20) if lib.log_n == 12 else (400 << 20)) for lib, _, evk, _ in rings]
    reqs = {}
    nreq = 60
    for i in range(nreq):
        r = int(rng.integers(0, 2))
        lib, orc, evk, ops = rings[r]
        lv = int(rng.integers(2, orc.L + 1))
        a = ops[int(rng.integers(0, 4))][:, :lv, :].contiguous()
        b = ops[int(rng.integers(0, 4))][:, :lv, :].contiguous()
        out = lib.empty(2, lv - 1, orc.N)
        reqs[i] = (r, lv, a, b, out)
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
    for i, (r, lv, a, b, out) in reqs.items():
        lib, orc, evk, ops = rings[r]
        _, alone = lib.he_mul(lv, a, b, evk, relin=False)
        assert np.array_equal(lib.to_host(out), lib.to_host(alone)), i
    srv.close()


def test_server_rejects_oversized_and_bad_levels():
    import paper_2003_04510_amd as P
    lib, orc = contexts("n12_L3")
    evk = lib.to_device(random_evk(orc, 3))
    srv = P.Server(hbm_budget=1 << 20, max_batch=4, max_inflight=1)
    with pytest.raises(P.HeError):
        srv.add_ring(lib, evk, 2 << 20)  # over the budget
    r = srv.add_ring(lib, evk, 1 << 20)  # too small for any request at N=2^12
    a = lib.to_device(synth.random_ciphertext(1, orc.q, orc.N))
    out = lib.empty(2, 2, orc.N)
    with pytest.raises(P.HeError):
        srv.submit(r, 0, 3, a, a, out)
    with pytest.raises(P.HeError):
        srv.submit(r, 1, 1, a, a, out)
    srv.close()
