"""GPU: key generation, encryption and decryption through the library match
the oracle bit for bit on the same random draws, and the decrypted HE Mul
result matches the FP64 product of the messages."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import contexts, log

pytestmark = pytest.mark.gpu


def _draws(w, orc):
    kd = synth.key_draws(w)
    a_pk = synth.uniform_limbs(synth.SEED_KEYS, orc.q, w.N, 30)
    a_evk = np.stack([synth.uniform_limbs(synth.SEED_KEYS, orc.moduli, w.N, 40 + j) for j in range(w.dnum)])
    return kd, a_pk, a_evk


@pytest.mark.parametrize("wname", ["n12_L3", "n16_L24", "n17_L45"])
def test_keys_encrypt_he_mul_decrypt(wname):
    w = synth.WORKLOADS[wname]
    lib, orc = contexts(wname)
    log("scheme", wname)
    kd, a_pk, a_evk = _draws(w, orc)
    pk_o, evk_o = orc.keygen(kd.s, kd.e_pk, kd.e_evk, a_pk, a_evk)
    pk, evk = lib.keygen(kd.s, kd.e_pk, kd.e_evk, a_pk, a_evk)
    assert np.array_equal(lib.to_host(pk), pk_o)
    assert np.array_equal(lib.to_host(evk), evk_o)
    scale = 2.0**w.log_scale
    level = w.L
    za, zb = synth.unit_disk(synth.SEED_MSG_A, w.slots), synth.unit_disk(synth.SEED_MSG_B, w.slots)
    cts, cts_o = [], []
    for z, seed in ((za, synth.SEED_ENC_A), (zb, synth.SEED_ENC_B)):
        ed = synth.enc_draws(w, seed)
        m = oracle.encode(z, scale, w.N)
        cts_o.append(orc.encrypt(level, m, ed.v, ed.e0, ed.e1, pk_o))
        cts.append(lib.encrypt(level, m, ed.v, ed.e0, ed.e1, pk))
        assert np.array_equal(lib.to_host(cts[-1]), cts_o[-1])
    relin, out = lib.he_mul(level, cts[0], cts[1], evk)
    want_relin, want_out = orc.he_mul(level, cts_o[0], cts_o[1], evk_o)
    assert np.array_equal(lib.to_host(relin), want_relin)
    assert np.array_equal(lib.to_host(out), want_out)
    # decryption through the library equals the oracle's
    m_lib = lib.to_host(lib.decrypt_limbs(level - 1, out, kd.s))
    assert np.array_equal(m_lib, orc.decrypt_limbs(level - 1, want_out, kd.s))
    # FP64 gates
    want = za * zb
    got_pre = oracle.decode(oracle.crt_centered(lib.to_host(lib.decrypt_limbs(level, relin, kd.s)), orc.q[:level]),
                            scale * scale)
    rel_pre = np.linalg.norm(got_pre - want) / np.linalg.norm(want)
    got = oracle.decode(oracle.crt_centered(m_lib, orc.q[:level - 1]), scale * scale / orc.q[level - 1])
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    err_inf = np.max(np.abs(got - want))
    log("  rel error before rescale 2^%.1f, after 2^%.1f, max abs 2^%.1f"
        % (np.log2(rel_pre), np.log2(rel), np.log2(err_inf)))
    assert rel_pre <= 2.0**-20
    if wname == "n16_L24":
        # scale after rescale is 2^80 / q_23 ~ 2^30: gate max error at the
        # analytic rescale-rounding bound 8 sqrt((1+h) N / 12) q_l / Delta^2
        bound = 8 * np.sqrt((1 + w.h) * w.N / 12.0) * orc.q[level - 1] / scale**2
        assert err_inf <= bound
    else:
        assert rel <= 2.0**-20
