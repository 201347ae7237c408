"""GPU rotation (automorphism + key switching) and rotation keys against the
oracle, bit for bit, through the C ABI."""
import numpy as np
import pytest

import synth
from gpu_common import contexts, log

pytestmark = pytest.mark.gpu


def _rot_key(lib, orc, w, rot, seed):
    kd = synth.key_draws(w)
    e_rk = synth.gaussian(seed, w.N, 16, w.dnum)
    a_rk = np.stack([synth.uniform_limbs(seed + 1, orc.moduli, w.N, j) for j in range(w.dnum)])
    want = orc.keygen_rot(kd.s, orc.galois(rot), e_rk, a_rk)
    got = lib.keygen_rot(kd.s, rot, e_rk, a_rk)
    return kd, want, got


@pytest.mark.parametrize("wname,level,rot", [
    ("n12_L3", 3, 1), ("n12_L3", 2, 5), ("n12_L3", 1, -1), ("n12_L3", 3, 1023),
    ("n16_L24", 24, 1), ("n16_L24", 7, -3), ("n16_L24", 13, 32767),
    ("n16_L24_d24", 9, 5), ("n12_L6_d1", 6, 2),
])
def test_rotate_matches_oracle(wname, level, rot):
    lib, orc = contexts(wname)
    w = synth.WORKLOADS[wname]
    log("rotate", wname, level, rot)
    kd, rk_want, rk = _rot_key(lib, orc, w, rot, 200 + (rot % 97))
    assert np.array_equal(lib.to_host(rk), rk_want)
    ct = synth.random_ciphertext(77 + level, orc.q[:level], orc.N)
    want = orc.rotate(level, ct, rk_want, orc.galois(rot))
    got = lib.to_host(lib.rotate(level, lib.to_device(ct), rk, rot))
    assert np.array_equal(got, want)


def test_rotate_errors():
    import paper_2003_04510_amd as P
    lib, orc = contexts("n12_L3")
    ct = lib.empty(2, 3, lib.N)
    rk = lib.empty(lib.dnum, 2, lib.L + lib.K, lib.N)
    with pytest.raises(P.HeError):
        lib.rotate(4, ct, rk, 1)          # level above L
    with pytest.raises(P.HeError):
        lib.rotate(3, ct, rk, 1, out=ct)  # output aliases the input
