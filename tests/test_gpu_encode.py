"""GPU encoding (Sec. III-A) and HE Add (Sec. III-B) against the oracle,
through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import contexts, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wname", ["n12_L3", "n16_L24"])
def test_encode_matches_oracle(wname):
    """Both sides round an FP64 FFT to integers; the FFTs sum in different
    orders, so a coefficient may differ by one where its exact value lies
    within rounding error of a half-integer.  Everything else is equal, and
    the coefficients decode to the slots."""
    lib, orc = contexts(wname)
    w = synth.WORKLOADS[wname]
    scale = 2.0**w.log_scale
    for n in (w.slots, 7):
        z = synth.unit_disk(31 + n, n)
        log("encode", wname, n)
        got = lib.to_host(lib.encode(z, scale)).view(np.int64)
        want = oracle.encode(z, scale, w.N)
        raw = oracle.encode(z, scale, w.N, rounded=False)
        diff = got - want
        assert np.abs(diff).max() <= 1
        # FP64 error of either FFT here is below 2^-11 in absolute value
        near_tie = np.abs(np.abs(raw - np.floor(raw)) - 0.5) < 1e-3
        assert np.all(near_tie[diff != 0]), int((diff != 0).sum())
        assert (diff != 0).sum() <= max(2, w.N // 1000)
        back = oracle.decode([int(x) for x in got], scale)
        assert np.abs(back[:n] - z).max() < 2.0**-25
        if n < len(back):  # slots past n encode zero
            assert np.abs(back[n:]).max() < 2.0**-25


def test_encode_errors():
    import paper_2003_04510_amd as P
    lib, _ = contexts("n12_L3")
    with pytest.raises(P.HeError):
        lib.encode(np.zeros(lib.N // 2 + 1, dtype=np.complex128), 2.0**40)
    with pytest.raises(P.HeError):
        lib.encode(np.zeros(4, dtype=np.complex128), -1.0)


@pytest.mark.parametrize("wname,level", [("n12_L3", 3), ("n16_L24", 24), ("n16_L24", 5)])
def test_he_add_bit_exact(wname, level):
    lib, orc = contexts(wname)
    c1 = synth.random_ciphertext(61, orc.q[:level], orc.N)
    c2 = synth.random_ciphertext(62, orc.q[:level], orc.N)
    c2[0, 0, :4] = np.array([q - 1 for q in orc.q[:1]] * 4, dtype=np.uint64)  # wrap-around
    want = orc.he_add(level, c1, c2)
    d1, d2 = lib.to_device(c1), lib.to_device(c2)
    assert np.array_equal(lib.to_host(lib.add(level, d1, d2)), want)
    # in place
    lib.add(level, d1, d2, out=d1)
    assert np.array_equal(lib.to_host(d1), want)


@pytest.mark.parametrize("wname,level", [("n12_L3", 3), ("n16_L24", 24), ("n16_L24", 2), ("n17_L45", 45)])
def test_decode_matches_oracle(wname, level):
    """GPU decoding of decrypted residues against the oracle's exact
    reconstruction + FFT (both FP64 at the end: equal to 2^-30 relative),
    and the whole encode -> encrypt -> decrypt -> decode chain on the GPU."""
    lib, orc = contexts(wname)
    w = synth.WORKLOADS[wname]
    scale = 2.0**w.log_scale
    kd = synth.key_draws(w)
    a_pk = synth.uniform_limbs(synth.SEED_KEYS, orc.q, w.N, 30)
    a_evk = np.stack([synth.uniform_limbs(synth.SEED_KEYS, orc.moduli, w.N, 40 + j) for j in range(w.dnum)])
    pk, _ = lib.keygen(kd.s, kd.e_pk, kd.e_evk, a_pk, a_evk)
    z = synth.unit_disk(41, w.slots)
    ed = synth.enc_draws(w, 42)
    ct = lib.encrypt(level, lib.to_host(lib.encode(z, scale)).view(np.int64), ed.v, ed.e0, ed.e1, pk)
    m = lib.decrypt_limbs(level, ct, kd.s)
    got = lib.decode(level, m, scale)
    want = oracle.decode(oracle.crt_centered(lib.to_host(m), orc.q[:level]), scale)
    assert np.abs(got - want).max() < 2.0**-30 * max(1.0, np.abs(want).max())
    assert np.abs(got - z).max() < 2.0**-20
    few = lib.decode(level, m, scale, 5)
    assert np.abs(few - got[:5]).max() == 0
