"""Shared helpers of the GPU parity tests (seeded inputs, oracle results)."""
import functools
import sys

import numpy as np
import pytest

import oracle
import synth


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_2003_04510_amd as P
    P.load_library()   # raises if the HIP library is missing: no fallback
    return P


@functools.lru_cache(maxsize=None)
def contexts(wname):
    """(library context, oracle context) for a workload."""
    P = need_gpu()
    w = synth.WORKLOADS[wname] if isinstance(wname, str) else wname
    lib = P.Context.for_workload(w)
    orc = oracle.Context.for_workload(w)
    assert lib.q == orc.q and lib.p == orc.p
    return lib, orc


def random_evk(orc, seed=10):
    """Uniform evk-shaped residues [dnum][2][L+K][N] (bit-exactness does not
    depend on evk structure)."""
    return np.stack([np.stack([synth.uniform_limbs(seed + j, orc.moduli, orc.N, u) for u in range(2)])
                     for j in range(orc.dnum)])
