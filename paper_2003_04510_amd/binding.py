"""ctypes binding of libhe_mi355x.so (argument marshalling only).

Ciphertexts, keys and workspaces are torch tensors on the GPU, dtype int64
holding the uint64 residues bit for bit.  Every call enqueues work on the
current torch stream of the context's device.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhe_mi355x.so")

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
vp = ctypes.c_void_p
u32 = ctypes.c_uint32

_lib = None


class HeError(RuntimeError):
    pass


class HeBusy(HeError):
    """HE_EBUSY: a bounded queue is full; retry after progress()."""


class BatchItem(ctypes.Structure):
    _fields_ = [("level", ctypes.c_uint32), ("ct1", vp), ("ct2", vp), ("relin", vp), ("out", vp)]


class BatchSched(ctypes.Structure):
    _fields_ = [("cols_tile", ctypes.c_uint32), ("blocks_tile", ctypes.c_uint32), ("chunks", ctypes.c_uint32),
                ("ip_fused", ctypes.c_uint32), ("radix", ctypes.c_uint32)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32),
                ("max_queue", ctypes.c_uint32), ("hold_us", ctypes.c_uint32)]


class HeCt(ctypes.Structure):
    _fields_ = [("data", vp), ("level", ctypes.c_uint32), ("scale", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint32), ("ms", ctypes.c_double),
                ("ops", ctypes.c_double), ("bytes", ctypes.c_double)]


def load_library():
    """Load the built HIP library; raise if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HeError("libhe_mi355x.so is not built (run paper_2003_04510_amd/build.py); "
                      "there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    L.he_gen_primes.argtypes = [u32, u32, u32, u64p, u32, u64p]
    L.he_ctx_create.argtypes = [u32, u32, u32, u32, u64p, u64p, ctypes.c_int, vp, ctypes.c_size_t,
                                ctypes.POINTER(vp)]
    L.he_ctx_create_w32.argtypes = L.he_ctx_create.argtypes
    L.he_ctx_word_bytes.argtypes = [vp]
    L.he_ctx_word_bytes.restype = u32
    L.he_mul32.argtypes = [vp, u32, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.he_ctx_device_bytes.argtypes = [u32, u32, u32, u32, u64p, u64p]
    L.he_ctx_device_bytes.restype = ctypes.c_size_t
    L.he_ctx_table_bytes.argtypes = [vp]
    L.he_ctx_table_bytes.restype = ctypes.c_size_t
    L.he_ct_import.argtypes = [vp, u64p, u32, ctypes.c_double, ctypes.POINTER(HeCt), vp]
    L.he_ct_export.argtypes = [vp, ctypes.POINTER(HeCt), u64p, vp]
    L.he_mul_ct.argtypes = [vp, vp, ctypes.POINTER(HeCt), ctypes.POINTER(HeCt), ctypes.POINTER(HeCt),
                            ctypes.POINTER(HeCt), vp, ctypes.c_size_t, vp]
    L.he_rescale_ct.argtypes = [vp, ctypes.POINTER(HeCt), ctypes.POINTER(HeCt), vp, ctypes.c_size_t, vp]
    L.he_ctx_destroy.argtypes = [vp]
    L.he_ctx_destroy.restype = None
    for f in ("he_ct_bytes", "he_workspace_bytes"):
        getattr(L, f).argtypes = [vp, u32]
        getattr(L, f).restype = ctypes.c_size_t
    for f in ("he_evk_bytes", "he_pk_bytes"):
        getattr(L, f).argtypes = [vp]
        getattr(L, f).restype = ctypes.c_size_t
    L.he_keygen.argtypes = [vp, i64p, i64p, u64p, i64p, u64p, vp, vp, vp, ctypes.c_size_t, vp]
    L.he_encrypt.argtypes = [vp, u32, i64p, i64p, i64p, i64p, vp, vp, vp, ctypes.c_size_t, vp]
    L.he_decrypt.argtypes = [vp, u32, vp, i64p, vp, vp, ctypes.c_size_t, vp]
    L.he_mul.argtypes = [vp, u32, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.he_rescale.argtypes = [vp, u32, vp, vp, vp, ctypes.c_size_t, vp]
    L.he_mul_noalloc.argtypes = [vp, u32, vp, vp, vp, vp, vp, vp]
    L.he_mul_noalloc_bytes.argtypes = [vp, u32]
    L.he_mul_noalloc_bytes.restype = ctypes.c_size_t
    L.he_ntt.argtypes = [vp, vp, u32, u32, ctypes.c_int, vp]
    L.he_ctx_info.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32),
                              ctypes.POINTER(u32), u64p]
    L.he_timing_enable.argtypes = [vp, ctypes.c_int, ctypes.c_char_p]
    L.he_timing_read.argtypes = [vp, ctypes.POINTER(KernelStat), u32, ctypes.POINTER(u32)]
    L.he_batch_workspace_bytes.argtypes = [vp, ctypes.POINTER(BatchItem), u32]
    L.he_batch_workspace_bytes.restype = ctypes.c_size_t
    L.he_batch_create.argtypes = [vp, ctypes.POINTER(BatchItem), u32, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.he_mul_batch.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    L.he_batch_destroy.argtypes = [vp]
    L.he_batch_destroy.restype = None
    L.he_batch_set_sched.argtypes = [vp, ctypes.POINTER(BatchSched), vp]
    L.he_batch_get_sched.argtypes = [vp, ctypes.POINTER(BatchSched)]
    L.he_batch_autotune.argtypes = [vp, vp, vp, u32, vp, ctypes.POINTER(BatchSched),
                                    ctypes.POINTER(ctypes.c_double)]
    L.he_batch_group_create.argtypes = [ctypes.POINTER(vp), u32, ctypes.POINTER(vp)]
    L.he_mul_batch_group.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int, vp]
    L.he_batch_group_destroy.argtypes = [vp]
    L.he_batch_group_destroy.restype = None
    L.he_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(vp)]
    L.he_server_arena_min_bytes.argtypes = [ctypes.POINTER(ServerCfg)]
    L.he_server_arena_min_bytes.restype = ctypes.c_size_t
    L.he_server_add_ring.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, ctypes.POINTER(u32)]
    L.he_server_submit.argtypes = [vp, u32, ctypes.c_uint64, u32, vp, vp, vp]
    L.he_server_progress.argtypes = [vp, ctypes.POINTER(u32)]
    L.he_server_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double), u32,
                                 ctypes.POINTER(u32)]
    L.he_server_stats.argtypes = [vp] + [ctypes.POINTER(ctypes.c_uint64)] * 4
    L.he_server_destroy.argtypes = [vp]
    L.he_server_destroy.restype = None
    L.he_big_ctx_create.argtypes = [u32, u32, ctypes.c_int, ctypes.POINTER(vp)]
    L.he_big_ctx_destroy.argtypes = [vp]
    L.he_big_ctx_destroy.restype = None
    L.he_big_info.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32), u64p]
    for f in ("he_big_ct_bytes", "he_big_evk_bytes", "he_big_evk_ntt_bytes", "he_big_workspace_bytes"):
        getattr(L, f).argtypes = [vp]
        getattr(L, f).restype = ctypes.c_size_t
    L.he_big_evk_prepare.argtypes = [vp, vp, vp, vp]
    L.he_big_mul.argtypes = [vp, u32, vp, vp, vp, vp, u32, vp, ctypes.c_size_t, vp]
    L.he_big_timing_enable.argtypes = [vp, ctypes.c_int]
    L.he_big_timing_read.argtypes = [vp, ctypes.POINTER(KernelStat), u32, ctypes.POINTER(u32)]
    L.he_encode.argtypes = [vp, vp, u32, ctypes.c_double, vp, vp, ctypes.c_size_t, vp]
    L.he_add.argtypes = [vp, u32, vp, vp, vp, vp]
    L.he_decode.argtypes = [vp, u32, vp, ctypes.c_double, u32, vp, vp, ctypes.c_size_t, vp]
    L.he_rotate.argtypes = [vp, u32, vp, vp, ctypes.c_int32, vp, vp, ctypes.c_size_t, vp]
    L.he_keygen_rot.argtypes = [vp, i64p, ctypes.c_int32, i64p, u64p, vp, vp, ctypes.c_size_t, vp]
    L.he_valu_peaks.argtypes = [ctypes.c_int, u32, u32, ctypes.POINTER(ctypes.c_double), vp]
    L.he_status_str.argtypes = [st]
    L.he_status_str.restype = ctypes.c_char_p
    L.he_last_error.restype = ctypes.c_char_p
    for f in ("he_gen_primes", "he_ctx_create", "he_keygen", "he_encrypt", "he_decrypt", "he_mul",
              "he_rescale", "he_ntt", "he_ctx_info", "he_timing_enable", "he_timing_read", "he_batch_create",
              "he_mul_batch", "he_server_create", "he_server_add_ring", "he_server_submit", "he_server_progress",
              "he_server_poll", "he_server_stats", "he_big_ctx_create", "he_big_info", "he_big_evk_prepare",
              "he_big_mul", "he_big_timing_enable", "he_big_timing_read", "he_encode", "he_decode", "he_add", "he_rotate",
              "he_keygen_rot", "he_ct_import", "he_ct_export", "he_mul_ct", "he_rescale_ct", "he_mul_noalloc", "he_valu_peaks", "he_ctx_create_w32", "he_mul32", "he_batch_group_create", "he_mul_batch_group"):
        getattr(L, f).restype = st
    _lib = L
    return L


def _check(code: int, what: str):
    if code != 0:
        L = load_library()
        msg = "%s: %s (%s)" % (what, L.he_status_str(code).decode(), L.he_last_error().decode())
        raise (HeBusy if code == -6 else HeError)(msg)


def _u64arr(xs):
    a = np.ascontiguousarray(np.array(list(xs), dtype=np.uint64))
    return a, a.ctypes.data_as(u64p)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(i64p)


def gen_primes(log_n: int, bits: int, count: int, exclude=()) -> list:
    out = np.zeros(max(count, 1), dtype=np.uint64)
    ex, exp = _u64arr(list(exclude) or [0])
    _check(load_library().he_gen_primes(log_n, bits, count, exp, len(exclude), out.ctypes.data_as(u64p)),
           "he_gen_primes")
    return [int(x) for x in out[:count]]


def workload_primes(w) -> tuple:
    """q_0..q_{L-1} of the listed sizes then K special primes, all distinct,
    each the largest prime of its size that is 1 mod 2N and not yet used."""
    used, q, p = [], [], []
    for b in w.q_bits:
        (x,) = gen_primes(w.log_n, b, 1, used)
        used.append(x)
        q.append(x)
    for _ in range(w.K):
        (x,) = gen_primes(w.log_n, w.p_bits, 1, used)
        used.append(x)
        p.append(x)
    return q, p


VALU_KINDS = ("mad_u64_u32", "mul_hi_u32", "mul_lo_u32", "fma_f64", "int32_full_rate")


def valu_peaks(device: int = 0, blocks: int = 8192, iters: int = 2048) -> dict:
    """Measured issue rates (lane-ops/s over the device) of the VALU
    instruction kinds in VALU_KINDS (he_valu_peaks)."""
    import torch
    out = (ctypes.c_double * len(VALU_KINDS))()
    st = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    _check(load_library().he_valu_peaks(device, blocks, iters, out, st), "he_valu_peaks")
    return dict(zip(VALU_KINDS, list(out)))


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else None


def _host(a, n: int, dtype, name: str):
    """A contiguous host copy of `a` with exactly n elements of dtype."""
    arr = np.ascontiguousarray(a, dtype=dtype)
    if arr.size != n:
        raise HeError("%s: expected %d elements, got %d" % (name, n, arr.size))
    return arr


class Context:
    """A device context: moduli, NTT and base-conversion tables on GPU `device`.
    word32=True stores residues as 32-bit words (every prime below 2^31):
    such a context runs he_mul32 only and its tensors are int32."""

    def __init__(self, log_n: int, q, p, dnum: int, device: int = 0, word32: bool = False):
        import torch
        self.torch = torch
        L = load_library()
        self.log_n, self.N = log_n, 1 << log_n
        self.q, self.p = [int(x) for x in q], [int(x) for x in p]
        self.L, self.K, self.dnum = len(self.q), len(self.p), dnum
        self.device = device
        qa, qp = _u64arr(self.q)
        pa, pp = _u64arr(self.p)
        nbytes = int(L.he_ctx_device_bytes(log_n, self.L, self.K, dnum, qp, pp))
        if nbytes == 0:
            raise HeError("he_ctx_device_bytes: invalid parameters")
        # the context's constant tables live in torch memory the binding owns
        self._tables = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=torch.device("cuda", device))
        h = vp()
        self.word32 = bool(word32)
        self.wdtype = torch.int32 if self.word32 else torch.int64
        create = L.he_ctx_create_w32 if self.word32 else L.he_ctx_create
        _check(create(log_n, self.L, self.K, dnum, qp, pp, device, vp(self._tables.data_ptr()),
                      self._tables.numel() * 8, ctypes.byref(h)), "he_ctx_create")
        self._h = h
        self._ws = {}

    @classmethod
    def for_workload(cls, w, device: int = 0, word32: bool = False):
        q, p = workload_primes(w)
        return cls(w.log_n, q, p, w.dnum, device, word32)

    def close(self):
        if getattr(self, "_h", None):
            load_library().he_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- sizes / memory
    @property
    def dev(self):
        return self.torch.device("cuda", self.device)

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.dev).cuda_stream)

    def ct_bytes(self, level):
        return int(load_library().he_ct_bytes(self._h, level))

    def evk_bytes(self):
        return int(load_library().he_evk_bytes(self._h))

    def table_bytes(self):
        return int(load_library().he_ctx_table_bytes(self._h))

    def workspace_bytes(self, level):
        return int(load_library().he_workspace_bytes(self._h, level))

    def empty(self, *shape):
        """Uninitialized residue words (int64, or int32 for 32-bit words)."""
        return self.torch.empty(shape, dtype=self.wdtype, device=self.dev)

    def _dev(self, t, words: int, name: str, dtype=None):
        """Check that t can be handed to the library as `words` 8-byte
        elements: a contiguous tensor on this context's GPU, of dtype int64
        (or `dtype`), with at least that many elements.  Raises HeError
        before any library call."""
        dtype = self.wdtype if dtype is None else dtype
        if t is None:
            raise HeError("%s: missing tensor" % name)
        if not t.is_cuda or t.device.index != self.dev.index:
            raise HeError("%s: tensor must live on cuda:%d" % (name, self.device))
        if t.dtype != dtype:
            raise HeError("%s: dtype %s, expected %s" % (name, t.dtype, dtype))
        if not t.is_contiguous():
            raise HeError("%s: tensor must be contiguous" % name)
        if t.numel() < words:
            raise HeError("%s: %d elements, need at least %d" % (name, t.numel(), words))
        return vp(t.data_ptr())

    def _ct(self, t, level: int, name: str):
        if level > self.L:
            raise HeError("%s: level %d not in [1, L = %d]" % (name, level, self.L))
        return self._dev(t, 2 * max(level, 0) * self.N, name)

    def workspace(self, level):
        """A cached workspace tensor large enough for `level`."""
        need = (self.workspace_bytes(level) + 7) // 8
        ws = self._ws.get("ws")
        if ws is None or ws.numel() < need:
            ws = self.torch.empty(need, dtype=self.torch.int64, device=self.dev)
            self._ws["ws"] = ws
        return ws

    def to_device(self, arr: np.ndarray):
        """Host residues (uint64 values) -> device words of this context."""
        if self.word32:
            a64 = np.ascontiguousarray(arr, dtype=np.uint64)
            if a64.size and int(a64.max()) >> 32:
                raise HeError("to_device: a residue does not fit a 32-bit word")
            a = a64.astype(np.uint32).view(np.int32)
        else:
            a = np.ascontiguousarray(arr, dtype=np.uint64).view(np.int64)
        return self.torch.from_numpy(a.copy()).to(self.dev)

    @staticmethod
    def to_host(t) -> np.ndarray:
        """Device words -> host residues as uint64 (32-bit words widened)."""
        h = t.detach().cpu().numpy()
        if h.dtype == np.int32:
            return h.view(np.uint32).astype(np.uint64)
        return h.view(np.uint64)

    # ---------------------------------------------------------- operations
    def keygen(self, s, e_pk, e_evk, a_pk, a_evk):
        """Keys from supplied random draws -> (pk [2][L][N], evk [dnum][2][L+K][N]) on the GPU."""
        L = load_library()
        N, nm = self.N, self.L + self.K
        pk = self.empty(2, self.L, N)
        evk = self.empty(self.dnum, 2, nm, N)
        ws = self.workspace(self.L)
        s_ = _host(s, N, np.int64, "keygen: s")
        e_ = _host(e_pk, N, np.int64, "keygen: e_pk")
        ee_ = _host(e_evk, self.dnum * N, np.int64, "keygen: e_evk")
        ap_ = _host(a_pk, self.L * N, np.uint64, "keygen: a_pk")
        ae_ = _host(a_evk, self.dnum * nm * N, np.uint64, "keygen: a_evk")
        _check(L.he_keygen(self._h, s_.ctypes.data_as(i64p), e_.ctypes.data_as(i64p), ap_.ctypes.data_as(u64p),
                           ee_.ctypes.data_as(i64p), ae_.ctypes.data_as(u64p), vp(pk.data_ptr()),
                           vp(evk.data_ptr()), vp(ws.data_ptr()), ws.numel() * 8, self._stream()), "he_keygen")
        return pk, evk

    def encrypt(self, level, m, v, e0, e1, pk):
        ct = self.empty(2, level, self.N)
        ws = self.workspace(level)
        arrs = [_host(x, self.N, np.int64, "encrypt: " + nm) for x, nm in ((m, "m"), (v, "v"), (e0, "e0"), (e1, "e1"))]
        _check(load_library().he_encrypt(self._h, level, *[x.ctypes.data_as(i64p) for x in arrs],
                                         self._dev(pk, 2 * self.L * self.N, "encrypt: pk"), vp(ct.data_ptr()),
                                         vp(ws.data_ptr()), ws.numel() * 8, self._stream()), "he_encrypt")
        return ct

    def encode(self, z, scale: float):
        """Complex slots (numpy, n <= N/2) -> int64 coefficients [N] on the GPU."""
        zz = np.ascontiguousarray(np.asarray(z, dtype=np.complex128)).view(np.float64)
        zd = self.torch.from_numpy(zz.copy()).to(self.dev)
        m = self.empty(self.N)
        ws = self.workspace(1)
        _check(load_library().he_encode(self._h, vp(zd.data_ptr()), len(zz) // 2, float(scale), vp(m.data_ptr()),
                                        vp(ws.data_ptr()), ws.numel() * 8, self._stream()), "he_encode")
        return m

    def keygen_rot(self, s, rot: int, e_rk, a_rk):
        """Rotation key of `rot` slots from supplied draws -> [dnum][2][L+K][N] on the GPU."""
        N, nm = self.N, self.L + self.K
        rk = self.empty(self.dnum, 2, nm, N)
        ws = self.workspace(self.L)
        s_ = _host(s, N, np.int64, "keygen_rot: s")
        e_ = _host(e_rk, self.dnum * N, np.int64, "keygen_rot: e_rk")
        a_ = _host(a_rk, self.dnum * nm * N, np.uint64, "keygen_rot: a_rk")
        _check(load_library().he_keygen_rot(self._h, s_.ctypes.data_as(i64p), int(rot), e_.ctypes.data_as(i64p),
                                            a_.ctypes.data_as(u64p), vp(rk.data_ptr()), vp(ws.data_ptr()),
                                            ws.numel() * 8, self._stream()), "he_keygen_rot")
        return rk

    def rotate(self, level, ct, rk, rot: int, out=None, ws=None):
        out = self.empty(2, level, self.N) if out is None else out
        ws = self.workspace(level) if ws is None else ws
        _check(load_library().he_rotate(self._h, level, self._ct(ct, level, "rotate: ct"),
                                        self._dev(rk, self.evk_bytes() // 8, "rotate: rk"), int(rot),
                                        self._ct(out, level, "rotate: out"),
                                        self._dev(ws, self.workspace_bytes(level) // 8, "rotate: workspace", self.torch.int64),
                                        ws.numel() * 8, self._stream()), "he_rotate")
        return out

    def decode(self, level, m_limbs, scale: float, n: int = None):
        """Coefficient-form residues [level][N] (device) -> n complex slots (numpy)."""
        n = self.N // 2 if n is None else n
        z = self.torch.empty(2 * max(n, 1), dtype=self.torch.float64, device=self.dev)
        ws = self.workspace(level)
        _check(load_library().he_decode(self._h, level, self._dev(m_limbs, level * self.N, "decode: m"), float(scale),
                                        n, vp(z.data_ptr()), vp(ws.data_ptr()), ws.numel() * 8, self._stream()),
               "he_decode")
        return z.cpu().numpy()[:2 * n].view(np.complex128)

    def add(self, level, ct1, ct2, out=None):
        out = self.empty(2, level, self.N) if out is None else out
        _check(load_library().he_add(self._h, level, self._ct(ct1, level, "add: ct1"), self._ct(ct2, level, "add: ct2"),
                                     self._ct(out, level, "add: out"), self._stream()), "he_add")
        return out

    def decrypt_limbs(self, level, ct, s):
        out = self.empty(level, self.N)
        ws = self.workspace(level)
        s_ = _host(s, self.N, np.int64, "decrypt: s")
        _check(load_library().he_decrypt(self._h, level, self._ct(ct, level, "decrypt: ct"), s_.ctypes.data_as(i64p),
                                         vp(out.data_ptr()), vp(ws.data_ptr()), ws.numel() * 8, self._stream()),
               "he_decrypt")
        return out

    def he_mul(self, level, ct1, ct2, evk, relin=True, rescale=True, ws=None, out_relin=None, out=None):
        """HE Mul; returns (relinearized ct or None, rescaled ct or None).
        32-bit-word contexts go through he_mul32."""
        if relin and out_relin is None:
            out_relin = self.empty(2, level, self.N)
        if rescale and out is None:
            out = self.empty(2, max(level - 1, 1), self.N)
        ws = self.workspace(level) if ws is None else ws
        fn = load_library().he_mul32 if self.word32 else load_library().he_mul
        _check(fn(self._h, level, self._ct(ct1, level, "he_mul: ct1"),
                                     self._ct(ct2, level, "he_mul: ct2"),
                                     self._dev(evk, self.evk_bytes() // 8, "he_mul: evk"),
                                     self._ct(out_relin, level, "he_mul: relin") if relin else None,
                                     self._ct(out, level - 1, "he_mul: out") if rescale else None,
                                     self._dev(ws, self.workspace_bytes(level) // 8, "he_mul: workspace", self.torch.int64), ws.numel() * 8,
                                     self._stream()), "he_mul")
        return (out_relin if relin else None), (out if rescale else None)

    def he_mul_noalloc(self, level, ct1, ct2, evk, out_relin=None, out=None):
        """he_mul_noalloc: HE Mul into caller tensors with the library's
        per-GPU scratch as workspace (no allocation in the library)."""
        _check(load_library().he_mul_noalloc(self._h, level, self._ct(ct1, level, "he_mul_noalloc: ct1"),
                                             self._ct(ct2, level, "he_mul_noalloc: ct2"),
                                             self._dev(evk, self.evk_bytes() // 8, "he_mul_noalloc: evk"),
                                             self._ct(out_relin, level, "he_mul_noalloc: relin")
                                             if out_relin is not None else None,
                                             self._ct(out, level - 1, "he_mul_noalloc: out") if out is not None
                                             else None, self._stream()), "he_mul_noalloc")
        return out_relin, out

    def noalloc_bytes(self, level):
        return int(load_library().he_mul_noalloc_bytes(self._h, level))

    def rescale(self, level, ct, out=None):
        out = self.empty(2, max(level - 1, 1), self.N) if out is None else out
        ws = self.workspace(level)
        _check(load_library().he_rescale(self._h, level, self._ct(ct, level, "rescale: ct"),
                                         self._ct(out, level - 1, "rescale: out"), vp(ws.data_ptr()),
                                         ws.numel() * 8, self._stream()), "he_rescale")
        return out

    # ---------------------------------------------------------- ciphertext descriptors
    def ct_import(self, host, level: int, scale: float):
        """Host residues [2][level][N] -> Ciphertext on the GPU (he_ct_import)."""
        h = _host(host, 2 * level * self.N, np.uint64, "ct_import: host")
        data = self.empty(2, level, self.N)
        ct = HeCt(data.data_ptr(), 0, 0.0)
        _check(load_library().he_ct_import(self._h, h.ctypes.data_as(u64p), level, float(scale), ctypes.byref(ct),
                                           self._stream()), "he_ct_import")
        return Ciphertext(data, ct.level, ct.scale)

    def ct_export(self, c: "Ciphertext") -> np.ndarray:
        """Ciphertext -> host residues [2][level][N] (he_ct_export)."""
        out = np.empty((2, c.level, self.N), dtype=np.uint64)
        ct = HeCt(self._ct(c.data, c.level, "ct_export").value, c.level, c.scale)
        _check(load_library().he_ct_export(self._h, ctypes.byref(ct), out.ctypes.data_as(u64p), self._stream()),
               "he_ct_export")
        return out

    def mul_ct(self, a: "Ciphertext", b: "Ciphertext", evk, relin: bool = True, rescale: bool = True):
        """he_mul_ct: returns (relinearized Ciphertext or None, rescaled Ciphertext or None)."""
        lv = a.level
        ws = self.workspace(lv)
        ca = HeCt(self._ct(a.data, lv, "mul_ct: a").value, a.level, a.scale)
        cb = HeCt(self._ct(b.data, b.level, "mul_ct: b").value, b.level, b.scale)
        r_t = self.empty(2, lv, self.N) if relin else None
        o_t = self.empty(2, max(lv - 1, 1), self.N) if rescale else None
        cr = HeCt(r_t.data_ptr(), 0, 0.0) if relin else None
        co = HeCt(o_t.data_ptr(), 0, 0.0) if rescale else None
        _check(load_library().he_mul_ct(self._h, self._dev(evk, self.evk_bytes() // 8, "mul_ct: evk"),
                                        ctypes.byref(ca), ctypes.byref(cb),
                                        ctypes.byref(cr) if cr is not None else None,
                                        ctypes.byref(co) if co is not None else None,
                                        vp(ws.data_ptr()), ws.numel() * 8, self._stream()), "he_mul_ct")
        return (Ciphertext(r_t, cr.level, cr.scale) if relin else None,
                Ciphertext(o_t, co.level, co.scale) if rescale else None)

    def rescale_ct(self, c: "Ciphertext"):
        ws = self.workspace(c.level)
        out = self.empty(2, max(c.level - 1, 1), self.N)
        ci = HeCt(self._ct(c.data, c.level, "rescale_ct").value, c.level, c.scale)
        co = HeCt(out.data_ptr(), 0, 0.0)
        _check(load_library().he_rescale_ct(self._h, ctypes.byref(ci), ctypes.byref(co), vp(ws.data_ptr()),
                                            ws.numel() * 8, self._stream()), "he_rescale_ct")
        return Ciphertext(out, co.level, co.scale)

    def timing(self, enable: bool, only: str = None):
        """Bracket library kernels with HIP events (all kinds, or only `only`)."""
        _check(load_library().he_timing_enable(self._h, int(enable), only.encode() if only else None),
               "he_timing_enable")

    def timing_read(self) -> dict:
        """{kind: (launches, ms, ops, bytes)} since the last read (synchronize first)."""
        arr = (KernelStat * 64)()
        n = u32(0)
        _check(load_library().he_timing_read(self._h, arr, 64, ctypes.byref(n)), "he_timing_read")
        return {arr[i].name.decode(): (arr[i].launches, arr[i].ms, arr[i].ops, arr[i].bytes)
                for i in range(min(n.value, 64))}

    def batch(self, items):
        """A batched HE Mul over items = [(level, ct1, ct2, relin_or_None, out_or_None), ...]."""
        return Batch(self, items)

    def ntt(self, data, first_mod: int, inverse: bool = False):
        """In-place transform of data [nlimbs][N]; limb r modulo modulus first_mod + r."""
        if data.numel() % self.N:
            raise HeError("ntt: size is not a multiple of N")
        nl = data.numel() // self.N
        _check(load_library().he_ntt(self._h, self._dev(data, nl * self.N, "ntt: data"), nl, first_mod, int(inverse),
                                     self._stream()), "he_ntt")
        return data


class Ciphertext:
    """A ciphertext on the GPU: data [2][level][N] (int64 tensor holding the
    uint64 residues), its level and its scale (he_ct)."""

    def __init__(self, data, level: int, scale: float):
        self.data, self.level, self.scale = data, int(level), float(scale)


class Batch:
    """Many HE Muls of one context as one sequence of batched stage kernels.
    The workspace is allocated here (torch) and kept alive with the batch."""

    def __init__(self, ctx: "Context", items):
        L = load_library()
        self.ctx = ctx
        self.items = list(items)
        arr = (BatchItem * len(self.items))()
        for i, (level, ct1, ct2, relin, out) in enumerate(self.items):
            tag = "batch item %d" % i
            arr[i] = BatchItem(level, ctx._ct(ct1, level, tag + " ct1").value, ctx._ct(ct2, level, tag + " ct2").value,
                               ctx._ct(relin, level, tag + " relin").value if relin is not None else None,
                               ctx._ct(out, level - 1, tag + " out").value if out is not None else None)
        self._arr = arr
        nbytes = int(L.he_batch_workspace_bytes(ctx._h, arr, len(self.items)))
        if nbytes == 0:
            raise HeError("he_batch_workspace_bytes: invalid items")
        self.ws = ctx.empty((nbytes + 7) // 8)
        h = vp()
        _check(L.he_batch_create(ctx._h, arr, len(self.items), vp(self.ws.data_ptr()), self.ws.numel() * 8,
                                 ctypes.byref(h)), "he_batch_create")
        self._h = h

    def run(self, evk, use_graph: bool = False):
        _check(load_library().he_mul_batch(self.ctx._h, self._h,
                                           self.ctx._dev(evk, self.ctx.evk_bytes() // 8, "batch: evk"), int(use_graph),
                                           self.ctx._stream()), "he_mul_batch")

    def set_sched(self, cols_tile: int, blocks_tile: int, chunks: int, ip_fused: int = 0, radix: int = 0):
        sc = BatchSched(cols_tile, blocks_tile, chunks, ip_fused, radix)
        _check(load_library().he_batch_set_sched(self._h, ctypes.byref(sc), self.ctx._stream()),
               "he_batch_set_sched")

    def sched(self):
        sc = BatchSched()
        _check(load_library().he_batch_get_sched(self._h, ctypes.byref(sc)), "he_batch_get_sched")
        return {"cols_tile": sc.cols_tile, "blocks_tile": sc.blocks_tile, "chunks": sc.chunks, "ip_fused": sc.ip_fused,
                "radix": sc.radix}

    def autotune(self, evk, reps: int = 3):
        """Time every candidate schedule (graph replays) and keep the
        fastest; returns (schedule, ms per replay)."""
        sc, ms = BatchSched(), ctypes.c_double()
        _check(load_library().he_batch_autotune(self.ctx._h, self._h,
                                                self.ctx._dev(evk, self.ctx.evk_bytes() // 8, "autotune: evk"), reps,
                                                self.ctx._stream(),
                                                ctypes.byref(sc), ctypes.byref(ms)), "he_batch_autotune")
        return ({"cols_tile": sc.cols_tile, "blocks_tile": sc.blocks_tile, "chunks": sc.chunks,
                 "ip_fused": sc.ip_fused, "radix": sc.radix}, ms.value)

    def close(self):
        if getattr(self, "_h", None):
            load_library().he_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGroup:
    """Batches of different contexts (ring sizes) run as one unit, each on a
    stream of its own, captured into one HIP graph (he_batch_group_*)."""

    def __init__(self, batches):
        self.batches = list(batches)
        if not self.batches:
            raise HeError("BatchGroup: no batches")
        dev = {b.ctx.device for b in self.batches}
        if len(dev) != 1:
            raise HeError("BatchGroup: batches on different devices")
        arr = (vp * len(self.batches))(*[b._h.value for b in self.batches])
        h = vp()
        _check(load_library().he_batch_group_create(arr, len(self.batches), ctypes.byref(h)), "he_batch_group_create")
        self._h = h

    def run(self, evks, use_graph: bool = True):
        if len(evks) != len(self.batches):
            raise HeError("BatchGroup.run: one evaluation key per batch")
        arr = (vp * len(evks))(*[b.ctx._dev(k, b.ctx.evk_bytes() // 8, "group evk %d" % i).value
                                 for i, (b, k) in enumerate(zip(self.batches, evks))])
        ctx0 = self.batches[0].ctx
        _check(load_library().he_mul_batch_group(self._h, arr, int(use_graph), ctx0._stream()), "he_mul_batch_group")

    def close(self):
        if getattr(self, "_h", None):
            load_library().he_batch_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching HE Mul server (the loop runs in the native library).
    The binding allocates each ring's arena (torch memory) and keeps every
    request's tensors alive until poll() has returned the request."""

    def __init__(self, hbm_budget: int, max_batch: int = 64, max_inflight: int = 2, max_queue: int = 0,
                 hold_us: int = 0):
        L = load_library()
        h = vp()
        self._cfg = ServerCfg(hbm_budget, max_batch, max_inflight, max_queue, hold_us)
        _check(L.he_server_create(ctypes.byref(self._cfg), ctypes.byref(h)), "he_server_create")
        self._h = h
        self._keep = []
        self._rings = []
        self._live = {}

    def arena_min_bytes(self) -> int:
        return int(load_library().he_server_arena_min_bytes(ctypes.byref(self._cfg)))

    def add_ring(self, ctx: "Context", evk, arena_bytes: int) -> int:
        ev = ctx._dev(evk, ctx.evk_bytes() // 8, "add_ring: evk")
        arena = ctx.empty((int(arena_bytes) + 7) // 8)
        rid = u32(0)
        _check(load_library().he_server_add_ring(self._h, ctx._h, ev, vp(arena.data_ptr()), arena.numel() * 8,
                                                 ctypes.byref(rid)), "he_server_add_ring")
        self._keep.append((ctx, evk, arena))
        self._rings.append(ctx)
        return rid.value

    def submit(self, ring: int, rid: int, level: int, ct1, ct2, out):
        if ring >= len(self._rings):
            raise HeError("submit: unknown ring %d" % ring)
        if rid in self._live:
            raise HeError("submit: request id %d is still in flight" % rid)
        ctx = self._rings[ring]
        _check(load_library().he_server_submit(self._h, ring, rid, level, ctx._ct(ct1, level, "submit: ct1"),
                                               ctx._ct(ct2, level, "submit: ct2"),
                                               ctx._ct(out, level - 1, "submit: out")), "he_server_submit")
        self._live[rid] = (ct1, ct2, out)

    def progress(self) -> int:
        n = u32(0)
        _check(load_library().he_server_progress(self._h, ctypes.byref(n)), "he_server_progress")
        return n.value

    def poll(self, maxn: int = 4096):
        ids = (ctypes.c_uint64 * maxn)()
        lat = (ctypes.c_double * maxn)()
        n = u32(0)
        _check(load_library().he_server_poll(self._h, ids, lat, maxn, ctypes.byref(n)), "he_server_poll")
        done = [(ids[i], lat[i]) for i in range(n.value)]
        for k, _ in done:
            self._live.pop(k, None)
        return done

    def stats(self) -> dict:
        v = [ctypes.c_uint64(0) for _ in range(4)]
        _check(load_library().he_server_stats(self._h, *[ctypes.byref(x) for x in v]), "he_server_stats")
        return dict(zip(("queued", "inflight", "batches", "completed"), [x.value for x in v]))

    def close(self):
        if getattr(self, "_h", None):
            load_library().he_server_destroy(self._h)   # waits for the rings' streams
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BigContext:
    """The paper's non-RNS HE Mul (power-of-two moduli, big-integer
    coefficients as [W][N] uint64 words) on GPU `device`."""

    def __init__(self, log_n: int, logQ: int, device: int = 0):
        import torch
        self.torch = torch
        L = load_library()
        self.log_n, self.N, self.logQ, self.device = log_n, 1 << log_n, logQ, device
        h = vp()
        _check(L.he_big_ctx_create(log_n, logQ, device, ctypes.byref(h)), "he_big_ctx_create")
        self._h = h
        np1, np2, W = u32(0), u32(0), u32(0)
        _check(L.he_big_info(h, ctypes.byref(np1), ctypes.byref(np2), ctypes.byref(W), None), "he_big_info")
        self.np1, self.np2, self.W = np1.value, np2.value, W.value
        self.W2 = (2 * logQ + 63) // 64
        pr = np.zeros(self.np2, dtype=np.uint64)
        _check(L.he_big_info(h, None, None, None, pr.ctypes.data_as(u64p)), "he_big_info")
        self.primes = [int(x) for x in pr]
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            load_library().he_big_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dev(self):
        return self.torch.device("cuda", self.device)

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.dev).cuda_stream)

    def empty(self, *shape):
        return self.torch.empty(shape, dtype=self.torch.int64, device=self.dev)

    def to_device(self, arr: np.ndarray):
        a = np.ascontiguousarray(arr, dtype=np.uint64).view(np.int64)
        return self.torch.from_numpy(a.copy()).to(self.dev)

    @staticmethod
    def to_host(t) -> np.ndarray:
        return t.detach().cpu().numpy().view(np.uint64)

    def workspace(self):
        need = int(load_library().he_big_workspace_bytes(self._h)) // 8
        if self._ws is None or self._ws.numel() < need:
            self._ws = self.empty(need)
        return self._ws

    def evk_prepare(self, evk):
        """evk [2][W2][N] words (below Q^2) -> NTT form [2][np2][N]."""
        out = self.empty(2, self.np2, self.N)
        _check(load_library().he_big_evk_prepare(self._h, vp(evk.data_ptr()), vp(out.data_ptr()), self._stream()),
               "he_big_evk_prepare")
        return out

    def he_mul(self, logq: int, ct1, ct2, evk_ntt, logp: int = 0, out=None, ws=None):
        """HE Mul at level 2^logq; rescaled by 2^logp when logp > 0.  -> [2][W][N]."""
        out = self.empty(2, self.W, self.N) if out is None else out
        ws = self.workspace() if ws is None else ws
        _check(load_library().he_big_mul(self._h, logq, vp(ct1.data_ptr()), vp(ct2.data_ptr()),
                                         vp(evk_ntt.data_ptr()), vp(out.data_ptr()), logp, vp(ws.data_ptr()),
                                         ws.numel() * 8, self._stream()), "he_big_mul")
        return out

    def timing(self, enable: bool):
        _check(load_library().he_big_timing_enable(self._h, int(enable)), "he_big_timing_enable")

    def timing_read(self) -> dict:
        arr = (KernelStat * 64)()
        n = u32(0)
        _check(load_library().he_big_timing_read(self._h, arr, 64, ctypes.byref(n)), "he_big_timing_read")
        return {arr[i].name.decode(): (arr[i].launches, arr[i].ms, arr[i].ops, arr[i].bytes)
                for i in range(min(n.value, 64))}
