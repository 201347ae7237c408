"""The oracle's pins catch plausible mistakes in the oracle itself.

Each case plants one mistake (a wrong sign, a dropped constant, a wrong root
or index) in a scratch copy of `oracle/he_oracle.c`, on the CPU, and runs
the CPU pins of `tests/test_oracle_pins.py` against that copy in a child
process: the pins must fail.  Nothing here touches the HIP library.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "he_oracle.c")

# (name, text of the oracle, its mistaken form[, line]): the text occurs
# once in the oracle, or on the given line
MUTATIONS = [
    ("ntt butterfly sign", "    a[h + k] = msub(lo, t, q);", "    a[h + k] = madd(lo, t, q);"),
    ("ntt root of the second half", "  ntt_split(a + h, h, E / 2 + N, q, pw, N);", "  ntt_split(a + h, h, E / 2, q, pw, N);"),
    ("intt without N^-1", "{ a[i] = mmul(a[i], ninv, q); g_intt_modmul++; }", "{ g_intt_modmul++; }"),
    ("intt wrong inverse root", "sinv = pw[2 * N - E / 2];", "sinv = pw[E / 2];"),
    ("tensor d1 term", "madd(mmul(a1, b2, q), mmul(a2, b1, q), q)", "madd(mmul(a1, b2, q), mmul(a2, b2, q), q)"),
    ("tensor d0", "      d[o] = mmul(b1, b2, q);", "      d[o] = mmul(b1, a2, q);"),
    ("mod up without the y scale", "mmul(x[(uint64_t)i * N + k], inv, qi)", "x[(uint64_t)i * N + k] % qi"),
    ("mod up constant with its own prime",
     "        for (uint32_t i2 = lo; i2 < hi; ++i2) if (i2 != i) prod = mmul(prod, c->mod[i2] % t, t);",
     "        for (uint32_t i2 = lo; i2 < hi; ++i2) prod = mmul(prod, c->mod[i2] % t, t);"),
    ("mod up own limbs zeroed", "        memcpy(dst, d2 + (uint64_t)e * N, sizeof(uint64_t) * N);",
     "        memset(dst, 0, sizeof(uint64_t) * N);"),
    ("inner product key polynomials swapped", "evk[(((uint64_t)j * 2 + u) * nm + mi) * N + k]",
     "evk[(((uint64_t)j * 2 + (1 - u)) * nm + mi) * N + k]"),
    ("mod down combine sign", "mmul(msub(ksu[(uint64_t)i * N + n], z[n], qi), pinv_q[i], qi)",
     "mmul(madd(ksu[(uint64_t)i * N + n], z[n], qi), pinv_q[i], qi)"),
    ("mod down without P^-1", "mmul(msub(ksu[(uint64_t)i * N + n], z[n], qi), pinv_q[i], qi)",
     "msub(ksu[(uint64_t)i * N + n], z[n], qi)"),
    ("mod down without (P/p_k)^-1", "yk[n] = mmul(yk[n], phat_inv[k], pk);", "yk[n] = yk[n] % pk;"),
    ("mod down without d", "        o[n] = madd(dd[n], md, qi);", "        o[n] = md;"),
    ("rescale without centring", "if (2 * (u128)r[n] < ql) s[n] = r[n] % qi;", "if (1) s[n] = r[n] % qi;"),
    ("rescale without q_l^-1", "o[n] = mmul(msub(ci[n], s[n], qi), qlinv, qi);", "o[n] = msub(ci[n], s[n], qi);"),
    ("rescale sign", "o[n] = mmul(msub(ci[n], s[n], qi), qlinv, qi);", "o[n] = mmul(madd(ci[n], s[n], qi), qlinv, qi);"),
    ("evk gadget without P", "if (in_digit) b = madd(b, mmul(Pm, mmul(sn[n], sn[n], m), m), m);",
     "if (in_digit) b = madd(b, mmul(sn[n], sn[n], m), m);"),
    ("evk gadget on every digit", "int in_digit = (i < L) && (i / c->alpha == j);", "int in_digit = (i < L);",
     "orc_keygen_evk"),
    ("automorphism without its sign flip", "else out[e - N] = in[k] ? m - in[k] : 0;", "else out[e - N] = in[k];"),
    ("root not the smallest", "if (cur < best) best = cur;", "if (cur > best) best = cur;"),
]


def _mutate(src, ent):
    name, a, b = ent[:3]
    if len(ent) == 4:  # the first occurrence after the named function
        start = src.index(ent[3])
        k = src.index(a, start)
        return src[:k] + b + src[k + len(a):]
    assert src.count(a) == 1, name
    return src.replace(a, b)


@pytest.mark.parametrize("ent", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(ent, tmp_path):
    src = open(SRC).read()
    mutated = _mutate(src, ent)
    assert mutated != src
    for d in ("oracle", "synth"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    os.makedirs(tmp_path / "tests")
    for f in ("conftest.py", "test_oracle_pins.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), tmp_path / "tests" / f)
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), tmp_path / "tests" / "golden")
    shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp_path / "pytest.ini")
    (tmp_path / "oracle" / "he_oracle.c").write_text(mutated)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py"], cwd=tmp_path, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "the pins pass with the mistake planted: %s\n%s" % (ent[0], r.stdout[-2000:])
    assert "failed" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
