"""CPU oracle for full-RNS HE Mul -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The HIP library never imports it and shares no code
with it.

Two layers:
  * `he_oracle.c` (built into liboracle.so): plain C with 128-bit `%`
    arithmetic for every modular product; NTT per Algorithm 3/4 of the paper.
  * this module: ctypes marshalling plus the pieces that need big integers or
    floating point -- CRT reconstruction (Python ints), CKKS encoding and
    decoding (numpy FFT as a library step), and tiny-N references used by
    the pins (schoolbook negacyclic convolution, closed-form NTT).

Parity unpinned: nothing here is compared against vectors from another
implementation (none exist for this path); every function is pinned by the
mathematical identities checked in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "he_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP over limbs only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_is_prime.argtypes = [ctypes.c_uint64]
        L.orc_is_prime.restype = ctypes.c_int
        L.orc_gen_primes.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, u64p, ctypes.c_uint32, u64p]
        L.orc_gen_primes.restype = ctypes.c_int
        L.orc_min_root.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
        L.orc_min_root.restype = ctypes.c_uint64
        L.orc_ctx_new.argtypes = [ctypes.c_uint32] * 4 + [u64p, u64p]
        L.orc_ctx_new.restype = ctypes.c_void_p
        L.orc_ctx_free.argtypes = [ctypes.c_void_p]
        L.orc_psi.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
        L.orc_psi.restype = ctypes.c_uint64
        L.orc_powers.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
        L.orc_powers.restype = u64p
        for f in ("orc_ntt", "orc_intt"):
            getattr(L, f).argtypes = [ctypes.c_void_p, ctypes.c_uint32, u64p]
        L.orc_tensor.argtypes = [ctypes.c_void_p, ctypes.c_uint32, u64p, u64p, u64p]
        L.orc_modup.argtypes = [ctypes.c_void_p, ctypes.c_uint32, u64p, u64p]
        L.orc_inner_product.argtypes = [ctypes.c_void_p, ctypes.c_uint32, u64p, u64p, u64p]
        L.orc_moddown_combine.argtypes = [ctypes.c_void_p, ctypes.c_uint32, u64p, u64p, u64p]
        L.orc_rescale.argtypes = [ctypes.c_void_p, ctypes.c_uint32, u64p, u64p]
        L.orc_he_mul.argtypes = [ctypes.c_void_p, ctypes.c_uint32, u64p, u64p, u64p, u64p, u64p]
        L.orc_num_digits.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
        L.orc_num_digits.restype = ctypes.c_uint32
        L.orc_keygen_pk.argtypes = [ctypes.c_void_p, i64p, i64p, u64p, u64p]
        L.orc_keygen_evk.argtypes = [ctypes.c_void_p, i64p, i64p, u64p, u64p]
        L.orc_encrypt.argtypes = [ctypes.c_void_p, ctypes.c_uint32, i64p, i64p, i64p, i64p, u64p, u64p]
        L.orc_decrypt_limbs.argtypes = [ctypes.c_void_p, ctypes.c_uint32, u64p, i64p, u64p]
        L.orc_automorphism.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, u64p, u64p]
        L.orc_keygen_rot.argtypes = [ctypes.c_void_p, i64p, ctypes.c_uint64, i64p, u64p, u64p]
        L.orc_rotate.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, u64p, u64p, u64p]
        for f in ("orc_counter_ntt", "orc_counter_intt"):
            getattr(L, f).restype = ctypes.c_uint64
        _lib = L
    return _lib


def _u(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(u64p)


def _i(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(i64p)


# ---------------------------------------------------------------- primes
def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's limb loops (timing only)."""
    return int(lib().orc_set_threads(int(n)))


def is_prime(n: int) -> bool:
    return bool(lib().orc_is_prime(n))


def gen_primes(log_n: int, bits: int, count: int, exclude=()) -> list:
    """The `count` largest primes < 2^bits that are 1 mod 2N (scan downward)."""
    ex = np.ascontiguousarray(np.array(list(exclude) or [0], dtype=np.uint64))
    out = np.zeros(max(count, 1), dtype=np.uint64)
    got = lib().orc_gen_primes(log_n, bits, count, _u(ex), len(exclude), _u(out))
    if got != count:
        raise ValueError("not enough primes")
    return [int(x) for x in out[:count]]


def workload_primes(w) -> tuple:
    """(q, p) for a workload: q_i of the listed sizes, K special primes of
    p_bits, all distinct; each size class takes the largest primes first."""
    used = []
    q = []
    for b in w.q_bits:
        (x,) = gen_primes(w.log_n, b, 1, exclude=used)
        used.append(x)
        q.append(x)
    p = []
    for _ in range(w.K):
        (x,) = gen_primes(w.log_n, w.p_bits, 1, exclude=used)
        used.append(x)
        p.append(x)
    return q, p


def min_root(q: int, log_n: int) -> int:
    return int(lib().orc_min_root(q, log_n))


def bitrev(x: int, bits: int) -> int:
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


# ---------------------------------------------------------------- context
class Context:
    """Moduli q_0..q_{L-1}, p_0..p_{K-1} and their NTT tables (oracle side)."""

    def __init__(self, log_n: int, q, p, dnum: int):
        self.log_n, self.N = log_n, 1 << log_n
        self.q, self.p = [int(x) for x in q], [int(x) for x in p]
        self.L, self.K, self.dnum = len(self.q), len(self.p), dnum
        self.alpha = -(-self.L // dnum)
        qa = np.array(self.q, dtype=np.uint64)
        pa = np.array(self.p or [0], dtype=np.uint64)
        self._h = lib().orc_ctx_new(log_n, self.L, self.K, dnum, _u(qa), _u(pa))

    @classmethod
    def for_workload(cls, w):
        q, p = workload_primes(w)
        return cls(w.log_n, q, p, w.dnum)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_ctx_free(self._h)
            self._h = None

    @property
    def moduli(self):
        return self.q + self.p

    def ext_moduli(self, level: int):
        """Extended basis E_l = q_0..q_{l-1}, p_0..p_{K-1}."""
        return self.q[:level] + self.p

    def num_digits(self, level: int) -> int:
        return -(-level // self.alpha)

    def digit(self, j: int, level: int):
        lo = j * self.alpha
        return list(range(lo, min(lo + self.alpha, level)))

    def psi(self, idx: int) -> int:
        return int(lib().orc_psi(self._h, idx))

    def powers(self, idx: int) -> np.ndarray:
        """psi^k mod modulus idx for 0 <= k < 2N (the transform's table)."""
        ptr = lib().orc_powers(self._h, idx)
        return np.ctypeslib.as_array(ptr, shape=(2 * self.N,)).copy()

    # -- transforms (idx indexes q_0..q_{L-1}, p_0..p_{K-1})
    def ntt(self, idx: int, a: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(a, dtype=np.uint64).copy()
        lib().orc_ntt(self._h, idx, _u(x))
        return x

    def intt(self, idx: int, a: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(a, dtype=np.uint64).copy()
        lib().orc_intt(self._h, idx, _u(x))
        return x

    # -- HE Mul steps
    def tensor(self, level, ct1, ct2):
        d = np.zeros((3, level, self.N), dtype=np.uint64)
        lib().orc_tensor(self._h, level, _u(_c(ct1)), _u(_c(ct2)), _u(d))
        return d

    def modup(self, level, d2):
        beta = self.num_digits(level)
        dt = np.zeros((beta, level + self.K, self.N), dtype=np.uint64)
        lib().orc_modup(self._h, level, _u(_c(d2)), _u(dt))
        return dt

    def inner_product(self, level, dt, evk):
        ks = np.zeros((2, level + self.K, self.N), dtype=np.uint64)
        lib().orc_inner_product(self._h, level, _u(_c(dt)), _u(_c(evk)), _u(ks))
        return ks

    def moddown_combine(self, level, ks, d):
        out = np.zeros((2, level, self.N), dtype=np.uint64)
        lib().orc_moddown_combine(self._h, level, _u(_c(ks)), _u(_c(d)), _u(out))
        return out

    def rescale(self, level, ct):
        out = np.zeros((2, level - 1, self.N), dtype=np.uint64)
        lib().orc_rescale(self._h, level, _u(_c(ct)), _u(out))
        return out

    def he_mul(self, level, ct1, ct2, evk, rescale=True):
        """Returns (relinearized ct at `level`, rescaled ct at level-1 or None)."""
        relin = np.zeros((2, level, self.N), dtype=np.uint64)
        out = np.zeros((2, level - 1, self.N), dtype=np.uint64) if (rescale and level >= 2) else None
        lib().orc_he_mul(self._h, level, _u(_c(ct1)), _u(_c(ct2)), _u(_c(evk)), _u(relin),
                         _u(out) if out is not None else None)
        return relin, out

    # -- keys, encryption, decryption (random draws are inputs)
    def keygen(self, s, e_pk, e_evk, a_pk, a_evk):
        pk = np.zeros((2, self.L, self.N), dtype=np.uint64)
        lib().orc_keygen_pk(self._h, _i(_ci(s)), _i(_ci(e_pk)), _u(_c(a_pk)), _u(pk))
        evk = np.zeros((self.dnum, 2, self.L + self.K, self.N), dtype=np.uint64)
        lib().orc_keygen_evk(self._h, _i(_ci(s)), _i(_ci(e_evk)), _u(_c(a_evk)), _u(evk))
        return pk, evk

    def encrypt(self, level, m_coeffs, v, e0, e1, pk):
        ct = np.zeros((2, level, self.N), dtype=np.uint64)
        lib().orc_encrypt(self._h, level, _i(_ci(m_coeffs)), _i(_ci(v)), _i(_ci(e0)), _i(_ci(e1)),
                          _u(_c(pk)), _u(ct))
        return ct

    # -- rotation (automorphism X -> X^g, g = 5^r mod 2N, then key switching)
    def galois(self, r: int) -> int:
        """g = 5^r mod 2N: slot j of sigma_g(m) is slot j + r of m."""
        return pow(5, r % (self.N // 2), 2 * self.N)

    def automorphism(self, level, ct, g):
        out = np.zeros((2, level, self.N), dtype=np.uint64)
        lib().orc_automorphism(self._h, level, g, _u(_c(ct)), _u(out))
        return out

    def keygen_rot(self, s, g, e_rk, a_rk):
        rk = np.zeros((self.dnum, 2, self.L + self.K, self.N), dtype=np.uint64)
        lib().orc_keygen_rot(self._h, _i(_ci(s)), g, _i(_ci(e_rk)), _u(_c(a_rk)), _u(rk))
        return rk

    def rotate(self, level, ct, rk, g):
        out = np.zeros((2, level, self.N), dtype=np.uint64)
        lib().orc_rotate(self._h, level, g, _u(_c(ct)), _u(_c(rk)), _u(out))
        return out

    def he_add(self, level, ct1, ct2):
        """HE Add (Sec. III-B): (c1 + c2) mod q_i limb by limb, [2][level][N]."""
        q = np.array(self.q[:level], dtype=np.uint64).reshape(1, level, 1)
        s = np.asarray(ct1, dtype=np.uint64) + np.asarray(ct2, dtype=np.uint64)
        return np.where(s >= q, s - q, s)

    def decrypt_limbs(self, level, ct, s):
        m = np.zeros((level, self.N), dtype=np.uint64)
        lib().orc_decrypt_limbs(self._h, level, _u(_c(ct)), _i(_ci(s)), _u(m))
        return m

    def decrypt(self, level, ct, s, scale, slots=None):
        m = self.decrypt_limbs(level, ct, s)
        coeffs = crt_centered(m, self.q[:level])
        return decode(coeffs, scale, slots)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def _ci(a):
    return np.ascontiguousarray(a, dtype=np.int64)


# ---------------------------------------------------------------- big integers
def crt(limbs, moduli) -> list:
    """CRT reconstruction: per coefficient the unique X in [0, prod moduli)."""
    Q = 1
    for m in moduli:
        Q *= int(m)
    terms = []
    for m in moduli:
        m = int(m)
        Qh = Q // m
        terms.append((Qh * pow(Qh % m, -1, m)) % Q)
    n = len(limbs[0])
    out = []
    for k in range(n):
        out.append(sum(int(limbs[i][k]) * terms[i] for i in range(len(moduli))) % Q)
    return out


def crt_centered(limbs, moduli) -> list:
    Q = 1
    for m in moduli:
        Q *= int(m)
    return [x - Q if 2 * x >= Q else x for x in crt(limbs, moduli)]


# ---------------------------------------------------------------- encoding
def slot_exponents(N: int) -> np.ndarray:
    """Slot j sits at the root zeta^{5^j mod 2N}, zeta = exp(i pi / N)."""
    e = np.empty(N // 2, dtype=np.int64)
    x = 1
    for j in range(N // 2):
        e[j] = x
        x = (x * 5) % (2 * N)
    return e


def encode(z: np.ndarray, scale: float, N: int, rounded: bool = True) -> np.ndarray:
    """Coefficients m with m(zeta^{5^j}) ~ scale*z_j, rounded to nearest: int64 [N]
    (float64 before the rounding when rounded is False).

    m_k = (2/N) Re sum_j scale z_j zeta^{-5^j k} written as one length-N FFT
    over the odd powers of zeta (all N of them, conjugates included)."""
    z = np.asarray(z, dtype=np.complex128)
    n = len(z)
    full = np.zeros(N // 2, dtype=np.complex128)
    full[:n] = z
    ex = slot_exponents(N)
    V = np.zeros(N, dtype=np.complex128)      # V[t] = value at zeta^{2t+1}
    V[(ex - 1) // 2] = scale * full
    V[((2 * N - ex) - 1) // 2] = scale * np.conj(full)
    k = np.arange(N)
    x = np.fft.fft(V) / N                       # = m_k zeta^k
    m = np.real(x * np.exp(-1j * np.pi * k / N))
    return np.rint(m).astype(np.int64) if rounded else m


def decode(coeffs, scale: float, slots=None) -> np.ndarray:
    """Evaluate the (centered) integer polynomial at zeta^{5^j}, divide by scale."""
    N = len(coeffs)
    m = np.array([float(c) for c in coeffs], dtype=np.float64)
    k = np.arange(N)
    V = N * np.fft.ifft(m * np.exp(1j * np.pi * k / N))   # V[t] = m(zeta^{2t+1})
    ex = slot_exponents(N)
    z = V[(ex - 1) // 2] / scale
    return z[:slots] if slots else z


# ---------------------------------------------------------------- tiny-N references
def schoolbook_negacyclic(a, b, q: int) -> list:
    """c = a*b in Z_q[X]/(X^N + 1) by the definition (O(N^2) Python ints)."""
    N = len(a)
    c = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                c[k] += int(a[i]) * int(b[j])
            else:
                c[k - N] -= int(a[i]) * int(b[j])
    return [x % q for x in c]


def ntt_closed_form(a, q: int, psi: int) -> list:
    """out[i] = sum_j a_j psi^{(2 bitrev(i) + 1) j} mod q (bit-reversed evaluation order)."""
    N = len(a)
    bits = N.bit_length() - 1
    out = []
    for i in range(N):
        r = pow(psi, 2 * bitrev(i, bits) + 1, q)
        out.append(sum(int(a[j]) * pow(r, j, q) for j in range(N)) % q)
    return out


def counters():
    return int(lib().orc_counter_ntt()), int(lib().orc_counter_intt())


def reset_counters():
    lib().orc_counter_reset()
