"""Thin Python binding of the C-ABI in include/ckkscnn.h.

Argument marshalling only: every homomorphic step runs in the HIP kernels of
libckkscnn.so.  PyTorch supplies device memory (ciphertext and plaintext
buffers are torch tensors on the GPU) and streams.  Loading fails loudly when
the library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libckkscnn.so")

CKC_ERRORS = {
    -1: "CKC_EINVAL", -2: "CKC_ELEVEL", -3: "CKC_ESCALE", -4: "CKC_ENOKEY",
    -5: "CKC_ENOMEM", -6: "CKC_EDEVICE", -7: "CKC_ESHAPE", -8: "CKC_EUNSUPPORTED",
}


class CkcError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn}: {CKC_ERRORS.get(code, code)}: {msg}")
        self.code = code


class ckc_ct(C.Structure):
    _fields_ = [("d", C.c_void_p), ("level", C.c_int32), ("npoly", C.c_int32), ("scale", C.c_double)]


class ckc_pt(C.Structure):
    _fields_ = [("d", C.c_void_p), ("level", C.c_int32), ("scale", C.c_double)]


class ckc_layout(C.Structure):
    _fields_ = [("block", C.c_int32), ("row_stride", C.c_int32), ("gap", C.c_int32), ("height", C.c_int32),
                ("width", C.c_int32), ("members", C.c_int32), ("flags", C.c_int32)]

    def as_tuple(self):
        return (self.block, self.row_stride, self.gap, self.height, self.width, self.members, self.flags)


_lib = None
_u64p = C.POINTER(C.c_uint64)
_i32p = C.POINTER(C.c_int32)
_dblp = C.POINTER(C.c_double)
_vp = C.c_void_p

# (name, restype, argtypes) for every entry point declared in include/ckkscnn.h
_SIGS = [
    ("ckc_last_error", C.c_char_p, []),
    ("ckc_ctx_create", C.c_int, [C.c_int, _u64p, C.c_int, _u64p, C.c_int, C.c_int, C.POINTER(_vp)]),
    ("ckc_ctx_destroy", C.c_int, [_vp]),
    ("ckc_ct_words", C.c_size_t, [_vp, C.c_int, C.c_int]),
    ("ckc_pt_words", C.c_size_t, [_vp, C.c_int]),
    ("ckc_ctx_root", C.c_uint64, [_vp, C.c_int]),
    ("ckc_ntt", C.c_int, [_vp, _vp, C.c_int, C.c_int, C.c_int, _vp]),
    ("ckc_keygen", C.c_int, [_vp, C.c_uint64, _i32p, C.c_int, C.POINTER(_vp), C.POINTER(_vp), _vp]),
    ("ckc_evk_add_rotations", C.c_int, [_vp, _vp, _vp, _i32p, C.c_int, _vp]),
    ("ckc_sk_destroy", C.c_int, [_vp]),
    ("ckc_evk_destroy", C.c_int, [_vp]),
    ("ckc_evk_bytes", C.c_size_t, [_vp]),
    ("ckc_encode", C.c_int, [_vp, _dblp, C.c_size_t, C.c_int, C.c_double, C.POINTER(ckc_pt), _vp]),
    ("ckc_encrypt", C.c_int, [_vp, _vp, C.POINTER(ckc_pt), C.c_uint64, C.POINTER(ckc_ct), _vp]),
    ("ckc_decrypt", C.c_int, [_vp, _vp, C.POINTER(ckc_ct), C.POINTER(ckc_pt), _vp]),
    ("ckc_decode", C.c_int, [_vp, C.POINTER(ckc_pt), _dblp, C.c_size_t, _vp]),
    ("ckc_add", C.c_int, [_vp, C.POINTER(ckc_ct), C.POINTER(ckc_ct), C.POINTER(ckc_ct), _vp]),
    ("ckc_sub", C.c_int, [_vp, C.POINTER(ckc_ct), C.POINTER(ckc_ct), C.POINTER(ckc_ct), _vp]),
    ("ckc_add_plain", C.c_int, [_vp, C.POINTER(ckc_ct), C.POINTER(ckc_pt), C.POINTER(ckc_ct), _vp]),
    ("ckc_add_const", C.c_int, [_vp, C.POINTER(ckc_ct), C.c_double, C.POINTER(ckc_ct), _vp]),
    ("ckc_mul_plain", C.c_int, [_vp, C.POINTER(ckc_ct), C.POINTER(ckc_pt), C.POINTER(ckc_ct), _vp]),
    ("ckc_tensor", C.c_int, [_vp, C.POINTER(ckc_ct), C.POINTER(ckc_ct), C.POINTER(ckc_ct), _vp]),
    ("ckc_relin", C.c_int, [_vp, _vp, C.POINTER(ckc_ct), C.POINTER(ckc_ct), _vp]),
    ("ckc_relin_noalloc", C.c_int, [_vp, _vp, C.POINTER(ckc_ct), C.POINTER(ckc_ct), _vp]),
    ("ckc_relin_noalloc_bytes", C.c_size_t, [_vp, C.c_int]),
    ("ckc_noalloc_capacity", C.c_size_t, []),
    ("ckc_rotate", C.c_int, [_vp, _vp, C.POINTER(ckc_ct), _i32p, C.c_int, C.POINTER(ckc_ct), _vp]),
    ("ckc_rescale", C.c_int, [_vp, C.POINTER(ckc_ct), C.POINTER(ckc_ct), _vp]),
    ("ckc_mod_drop", C.c_int, [_vp, C.POINTER(ckc_ct), C.c_int, C.POINTER(ckc_ct), _vp]),
    ("ckc_rescale_many", C.c_int, [_vp, C.POINTER(ckc_ct), C.c_int, C.POINTER(ckc_ct), _vp]),
    ("ckc_add_many", C.c_int, [_vp, C.POINTER(ckc_ct), C.POINTER(ckc_ct), C.c_int, C.POINTER(ckc_ct), _vp]),
    ("ckc_rotate_many", C.c_int, [_vp, _vp, C.POINTER(ckc_ct), C.c_int, _i32p, C.c_int, C.POINTER(ckc_ct), _vp]),
    ("ckc_mul_relin_many", C.c_int, [_vp, _vp, C.POINTER(ckc_ct), C.POINTER(ckc_ct), C.c_int, C.POINTER(ckc_ct),
                                     _vp]),
    ("ckc_mac_plain_many", C.c_int, [_vp, C.POINTER(ckc_ct), C.POINTER(ckc_pt), C.c_int, C.c_int,
                                     C.POINTER(ckc_ct), _vp]),
    ("ckc_layer_create_conv", C.c_int, [_vp, C.POINTER(ckc_layout), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                        _dblp, C.POINTER(C.c_uint16), _dblp, C.c_int, C.c_double, C.c_double,
                                        C.POINTER(_vp), _vp]),
    ("ckc_layer_create_conv_ex", C.c_int, [_vp, C.POINTER(ckc_layout), C.c_int, C.c_int, C.c_int, C.c_int,
                                           C.c_int, _dblp, C.POINTER(C.c_uint16), _dblp, C.c_int, C.c_double,
                                           C.c_double, C.c_int, C.POINTER(_vp), _vp]),
    ("ckc_eval_conv", C.c_int, [_vp, _vp, _vp, C.POINTER(ckc_ct), C.c_int, C.POINTER(ckc_ct), _vp]),
    ("ckc_layer_create_act", C.c_int, [_vp, C.POINTER(ckc_layout), C.c_int, _dblp, _dblp, C.c_double, C.c_int,
                                       C.c_double, C.POINTER(_vp), _vp]),
    ("ckc_eval_quad_act", C.c_int, [_vp, _vp, _vp, C.POINTER(ckc_ct), C.c_int, C.POINTER(ckc_ct), _vp]),
    ("ckc_layer_create_dense", C.c_int, [_vp, C.POINTER(ckc_layout), C.c_int, C.c_int, _dblp, _dblp, C.c_int,
                                         C.c_double, C.c_double, C.POINTER(_vp), _vp]),
    ("ckc_layer_create_dense_spatial", C.c_int, [_vp, C.POINTER(ckc_layout), C.c_int, C.c_int, _dblp, _dblp,
                                                 C.c_int, C.c_double, C.c_double, C.POINTER(_vp), _vp]),
    ("ckc_eval_dense", C.c_int, [_vp, _vp, _vp, C.POINTER(ckc_ct), C.c_int, C.POINTER(ckc_ct), _vp]),
    ("ckc_eval_avgpool2", C.c_int, [_vp, _vp, C.POINTER(ckc_layout), C.POINTER(ckc_ct), C.c_int,
                                    C.POINTER(ckc_ct), _vp]),
    ("ckc_layer_steps", C.c_int, [_vp, _i32p, C.c_int]),
    ("ckc_layer_out_layout", C.c_int, [_vp, C.POINTER(ckc_layout)]),
    ("ckc_layer_bytes", C.c_size_t, [_vp]),
    ("ckc_layer_destroy", C.c_int, [_vp]),
    ("ckc_prof_enable", C.c_int, [C.c_int]),
    ("ckc_prof_query", C.c_int, [C.c_char_p, C.POINTER(C.c_int64), _dblp, _dblp, _dblp]),
    ("ckc_variant_enable", C.c_int, [C.c_int]),
    ("ckc_variant_count", C.c_int, [C.c_char_p, C.POINTER(C.c_int64)]),
    ("ckc_variant_list", C.c_int, [C.c_char_p, C.c_size_t]),
    ("ckc_evk_group_create", C.c_int, [C.POINTER(_vp), C.c_int, _i32p, C.c_int, C.POINTER(_vp)]),
    ("ckc_tune_set", C.c_int, [C.c_char_p, C.c_int]),
    ("ckc_tune_get", C.c_int, [C.c_char_p, C.POINTER(C.c_int)]),
    ("ckc_stream_release", C.c_int, [C.c_void_p]),
    ("ckc_stream_reserve", C.c_int, [C.c_void_p, C.c_size_t]),
    ("ckc_ct_bytes", C.c_size_t, [C.c_void_p, C.c_int, C.c_int]),
    ("ckc_encode_encrypt_image", C.c_int, [C.c_void_p, C.c_void_p, _dblp, C.c_int, C.c_int, C.c_int, C.c_int,
                                           C.c_int, C.c_int, C.c_int, C.c_double, C.c_uint64, C.c_void_p,
                                           C.c_void_p]),
    ("ckc_set_test_fault", C.c_int, [C.c_int, C.c_int]),
    ("ckc_batch_plan", C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_void_p)]),
    ("ckc_batch_plan_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]),
    ("ckc_batch_plan_destroy", C.c_int, [C.c_void_p]),
    ("ckc_batch_run", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int,
                                C.POINTER(C.c_void_p), C.c_void_p]),
]


def exported_names() -> list[str]:
    return [n for n, _, _ in _SIGS]


def lib():
    """Load libckkscnn.so (raises if it has not been built).

    torch is imported first: its wheel carries its own HIP and HSA runtime
    libraries, which it must load before the library brings in the system
    ones (loaded the other way round, torch finds no GPU)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        import torch  # noqa: F401  (load order, see above)
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(fn: str, rc: int):
    if rc != 0:
        raise CkcError(fn, rc, lib().ckc_last_error().decode(errors="replace"))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


@dataclass
class Ciphertext:
    """Device ciphertext: `buf` is a torch int64 tensor holding [npoly][level+1][N] words."""
    buf: object
    level: int
    npoly: int
    scale: float

    def c(self) -> ckc_ct:
        return ckc_ct(self.buf.data_ptr(), self.level, self.npoly, self.scale)

    def update(self, s: ckc_ct):
        self.level, self.npoly, self.scale = int(s.level), int(s.npoly), float(s.scale)


@dataclass
class Plaintext:
    buf: object
    level: int
    scale: float

    def c(self) -> ckc_pt:
        return ckc_pt(self.buf.data_ptr(), self.level, self.scale)


class Context:
    """ckc_ctx: parameters and device tables."""

    def __init__(self, logN: int, q, p, alpha: int, device: str = "cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.logN, self.N = int(logN), 1 << int(logN)
        self.q, self.p, self.alpha = [int(x) for x in q], [int(x) for x in p], int(alpha)
        qa = (C.c_uint64 * len(self.q))(*self.q)
        pa = (C.c_uint64 * len(self.p))(*self.p)
        h = _vp()
        _check("ckc_ctx_create", lib().ckc_ctx_create(self.logN, qa, len(self.q), pa, len(self.p), self.alpha, C.byref(h)))
        self.h = h

    @classmethod
    def from_params(cls, ps, device: str = "cuda") -> "Context":
        return cls(ps.logN, ps.q, ps.p, ps.alpha, device)

    def close(self):
        if getattr(self, "h", None):
            lib().ckc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------- buffers
    def ct_words(self, level: int, npoly: int = 2) -> int:
        return int(lib().ckc_ct_words(self.h, level, npoly))

    def new_ct(self, level: int, npoly: int = 2, scale: float = 1.0) -> Ciphertext:
        buf = self.torch.empty(self.ct_words(level, npoly), dtype=self.torch.int64, device=self.device)
        return Ciphertext(buf, level, npoly, scale)

    def new_pt(self, level: int, scale: float = 1.0) -> Plaintext:
        buf = self.torch.empty(int(lib().ckc_pt_words(self.h, level)), dtype=self.torch.int64, device=self.device)
        return Plaintext(buf, level, scale)

    def upload_words(self, arr: np.ndarray):
        a = np.ascontiguousarray(arr, dtype=np.uint64).reshape(-1).view(np.int64)
        return self.torch.from_numpy(a.copy()).to(self.device)

    @staticmethod
    def download_words(buf) -> np.ndarray:
        return buf.detach().cpu().numpy().view(np.uint64).copy()

    def root(self, t: int) -> int:
        return int(lib().ckc_ctx_root(self.h, t))

    # --------------------------------------------------------- NTT
    def ntt(self, buf, n_blocks: int, n_limbs: int, inverse: bool, stream=None):
        _check("ckc_ntt", lib().ckc_ntt(self.h, buf.data_ptr(), n_blocks, n_limbs, int(inverse), _stream(stream)))

    def ct_from_coeff(self, data: np.ndarray, level: int, scale: float) -> Ciphertext:
        """Upload a coefficient-form ciphertext [npoly][level+1][N] and move it to NTT form."""
        npoly = data.shape[0]
        buf = self.upload_words(data)
        self.ntt(buf, npoly, level + 1, False)
        return Ciphertext(buf, level, npoly, scale)

    def pt_from_coeff(self, data: np.ndarray, level: int, scale: float) -> Plaintext:
        buf = self.upload_words(data[:level + 1])
        self.ntt(buf, 1, level + 1, False)
        return Plaintext(buf, level, scale)

    def ct_to_coeff(self, ct: Ciphertext) -> np.ndarray:
        tmp = ct.buf.clone()
        self.ntt(tmp, ct.npoly, ct.level + 1, True)
        self.torch.cuda.synchronize()
        return self.download_words(tmp).reshape(ct.npoly, ct.level + 1, self.N)

    def pt_to_coeff(self, pt: Plaintext) -> np.ndarray:
        tmp = pt.buf.clone()
        self.ntt(tmp, 1, pt.level + 1, True)
        self.torch.cuda.synchronize()
        return self.download_words(tmp).reshape(pt.level + 1, self.N)

    # --------------------------------------------------------- keys
    def keygen(self, seed: int, steps=(), stream=None):
        st = np.ascontiguousarray(np.array(list(steps), dtype=np.int32))
        sk, evk = _vp(), _vp()
        _check("ckc_keygen", lib().ckc_keygen(self.h, seed, st.ctypes.data_as(_i32p), len(st), C.byref(sk),
                                              C.byref(evk), _stream(stream)))
        return KeyPair(self, sk, evk)

    # --------------------------------------------------------- client
    def encode(self, slots, level: int, scale: float, out: Plaintext | None = None, stream=None) -> Plaintext:
        z = np.ascontiguousarray(np.asarray(slots, dtype=np.float64))
        pt = out or self.new_pt(level, scale)
        s = pt.c()
        _check("ckc_encode", lib().ckc_encode(self.h, z.ctypes.data_as(_dblp), len(z), level, float(scale),
                                              C.byref(s), _stream(stream)))
        pt.level, pt.scale = int(s.level), float(s.scale)
        return pt

    def ct_bytes(self, level: int, npoly: int = 2) -> int:
        return int(lib().ckc_ct_bytes(self.h, level, npoly))

    def encode_encrypt_image(self, keys: "KeyPair", chw, members: int, block: int, row_stride: int, level: int,
                             scale: float, stream_id: int, stream=None) -> list:
        """HW-layout packing and encryption of one image [C][H][W] in one call:
        ciphertext c uses PRNG stream stream_id + c."""
        x = np.ascontiguousarray(np.asarray(chw, dtype=np.float64))
        Cn, H, W = x.shape
        outs = [self.new_ct(level, 2, scale) for _ in range(Cn)]
        arr = (ckc_ct * Cn)(*[o.c() for o in outs])
        _check("ckc_encode_encrypt_image",
               lib().ckc_encode_encrypt_image(self.h, keys.sk, x.ctypes.data_as(_dblp), Cn, H, W, members, block,
                                              row_stride, level, float(scale), int(stream_id), arr,
                                              _stream(stream)))
        for o, a in zip(outs, arr):
            o.update(a)
        return outs

    def encrypt(self, keys: "KeyPair", pt: Plaintext, stream_id: int, out: Ciphertext | None = None,
                stream=None) -> Ciphertext:
        ct = out or self.new_ct(pt.level, 2, pt.scale)
        s, p = ct.c(), pt.c()
        _check("ckc_encrypt", lib().ckc_encrypt(self.h, keys.sk, C.byref(p), stream_id, C.byref(s), _stream(stream)))
        ct.update(s)
        return ct

    def decrypt(self, keys: "KeyPair", ct: Ciphertext, stream=None) -> Plaintext:
        pt = self.new_pt(ct.level, ct.scale)
        s, p = ct.c(), pt.c()
        _check("ckc_decrypt", lib().ckc_decrypt(self.h, keys.sk, C.byref(s), C.byref(p), _stream(stream)))
        pt.level, pt.scale = int(p.level), float(p.scale)
        return pt

    def decode(self, pt: Plaintext, n: int | None = None, stream=None) -> np.ndarray:
        n = self.N // 2 if n is None else n
        out = np.empty(n, dtype=np.float64)
        p = pt.c()
        _check("ckc_decode", lib().ckc_decode(self.h, C.byref(p), out.ctypes.data_as(_dblp), n, _stream(stream)))
        return out

    # --------------------------------------------------------- arithmetic
    def _binop(self, fn, a: Ciphertext, b: Ciphertext, out: Ciphertext | None, npoly_out: int, stream):
        out = out or self.new_ct(a.level, npoly_out, a.scale)
        sa, sb, so = a.c(), b.c(), out.c()
        _check(fn, getattr(lib(), fn)(self.h, C.byref(sa), C.byref(sb), C.byref(so), _stream(stream)))
        out.update(so)
        return out

    def add(self, a, b, out=None, stream=None):
        return self._binop("ckc_add", a, b, out, max(a.npoly, b.npoly), stream)

    def sub(self, a, b, out=None, stream=None):
        return self._binop("ckc_sub", a, b, out, max(a.npoly, b.npoly), stream)

    def tensor(self, a, b, out=None, stream=None):
        return self._binop("ckc_tensor", a, b, out, 3, stream)

    def add_plain(self, a: Ciphertext, p: Plaintext, out=None, stream=None):
        out = out or self.new_ct(a.level, a.npoly, a.scale)
        sa, sp, so = a.c(), p.c(), out.c()
        _check("ckc_add_plain", lib().ckc_add_plain(self.h, C.byref(sa), C.byref(sp), C.byref(so), _stream(stream)))
        out.update(so)
        return out

    def mul_plain(self, a: Ciphertext, p: Plaintext, out=None, stream=None):
        out = out or self.new_ct(a.level, a.npoly, a.scale)
        sa, sp, so = a.c(), p.c(), out.c()
        _check("ckc_mul_plain", lib().ckc_mul_plain(self.h, C.byref(sa), C.byref(sp), C.byref(so), _stream(stream)))
        out.update(so)
        return out

    def add_const(self, a: Ciphertext, value: float, out=None, stream=None):
        out = out or self.new_ct(a.level, a.npoly, a.scale)
        sa, so = a.c(), out.c()
        _check("ckc_add_const", lib().ckc_add_const(self.h, C.byref(sa), float(value), C.byref(so), _stream(stream)))
        out.update(so)
        return out

    def relin(self, keys: "KeyPair", a: Ciphertext, out=None, stream=None):
        out = out or self.new_ct(a.level, 2, a.scale)
        sa, so = a.c(), out.c()
        _check("ckc_relin", lib().ckc_relin(self.h, keys.evk, C.byref(sa), C.byref(so), _stream(stream)))
        out.update(so)
        return out

    def relin_noalloc(self, keys: "KeyPair", a: Ciphertext, out: Ciphertext, stream=None):
        """ckc_relin without device allocation (scratch in the library's
        static array); `out` must be given."""
        sa, so = a.c(), out.c()
        _check("ckc_relin_noalloc",
               lib().ckc_relin_noalloc(self.h, keys.evk, C.byref(sa), C.byref(so), _stream(stream)))
        out.update(so)
        return out

    def rotate(self, keys: "KeyPair", a: Ciphertext, steps, outs=None, stream=None):
        steps = list(steps)
        outs = outs or [self.new_ct(a.level, 2, a.scale) for _ in steps]
        arr = (ckc_ct * len(steps))(*[o.c() for o in outs])
        st = (C.c_int32 * len(steps))(*steps)
        sa = a.c()
        _check("ckc_rotate", lib().ckc_rotate(self.h, keys.evk, C.byref(sa), st, len(steps), arr, _stream(stream)))
        for o, s in zip(outs, arr):
            o.update(s)
        return outs

    def rescale(self, a: Ciphertext, out=None, stream=None):
        out = out or self.new_ct(max(a.level - 1, 0), a.npoly, a.scale)
        sa, so = a.c(), out.c()
        _check("ckc_rescale", lib().ckc_rescale(self.h, C.byref(sa), C.byref(so), _stream(stream)))
        out.update(so)
        return out

    def mod_drop(self, a: Ciphertext, to_level: int, out=None, stream=None):
        out = out or self.new_ct(to_level, a.npoly, a.scale)
        sa, so = a.c(), out.c()
        _check("ckc_mod_drop", lib().ckc_mod_drop(self.h, C.byref(sa), to_level, C.byref(so), _stream(stream)))
        out.update(so)
        return out


class KeyGroup:
    """A key group (ckc_evk_group_create): the key set of every image of a
    batched layer call.  keys: KeyPair objects (kept alive here); key_of_img:
    index into keys per image.  Usable wherever the layer calls take keys."""

    def __init__(self, keys, key_of_img):
        self.keys = list(keys)
        self.key_of_img = [int(k) for k in key_of_img]
        arr = (_vp * len(self.keys))(*[k.evk for k in self.keys])
        idx = (C.c_int32 * len(self.key_of_img))(*self.key_of_img)
        h = _vp()
        _check("ckc_evk_group_create",
               lib().ckc_evk_group_create(arr, len(self.keys), idx, len(self.key_of_img), C.byref(h)))
        self.evk = h

    def slice(self, i, j) -> "KeyGroup":
        """The group of images i .. j - 1."""
        return KeyGroup(self.keys, self.key_of_img[i:j])

    def evk_bytes(self) -> int:
        return 0

    def __del__(self):
        try:
            if getattr(self, "evk", None):
                lib().ckc_evk_destroy(self.evk)
                self.evk = None
        except Exception:
            pass


class KeyPair:
    """ckc_sk + ckc_evk handles from ckc_keygen."""

    def __init__(self, ctx: Context, sk, evk):
        self.ctx, self.sk, self.evk = ctx, sk, evk

    def add_rotations(self, steps, stream=None):
        st = (C.c_int32 * len(steps))(*steps)
        _check("ckc_evk_add_rotations", lib().ckc_evk_add_rotations(self.ctx.h, self.sk, self.evk, st, len(steps),
                                                                    _stream(stream)))

    def evk_bytes(self) -> int:
        return int(lib().ckc_evk_bytes(self.evk))

    def close(self):
        if self.sk:
            lib().ckc_sk_destroy(self.sk)
            self.sk = None
        if self.evk:
            lib().ckc_evk_destroy(self.evk)
            self.evk = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- layers
def _dbl(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(_dblp)


def _ct_array(cts):
    arr = (ckc_ct * len(cts))(*[c.c() for c in cts])
    return arr


def _update_all(cts, arr):
    for c, s in zip(cts, arr):
        c.update(s)


class Layer:
    """ckc_layer handle (conv, activation or dense)."""

    def __init__(self, ctx: Context, h, kind: str):
        self.ctx, self.h, self.kind = ctx, h, kind

    def steps(self) -> list[int]:
        n = lib().ckc_layer_steps(self.h, None, 0)
        buf = (C.c_int32 * max(n, 1))()
        lib().ckc_layer_steps(self.h, buf, n)
        return [int(buf[i]) for i in range(n)]

    def out_layout(self) -> ckc_layout:
        L = ckc_layout()
        _check("ckc_layer_out_layout", lib().ckc_layer_out_layout(self.h, C.byref(L)))
        return L

    def nbytes(self) -> int:
        return int(lib().ckc_layer_bytes(self.h))

    def close(self):
        if self.h:
            lib().ckc_layer_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


LAYOUT_SLICE_SHARED = 1  # CKC_LAYOUT_SLICE_SHARED


def make_layout(block, row_stride, gap, height, width, members, flags=0) -> ckc_layout:
    return ckc_layout(int(block), int(row_stride), int(gap), int(height), int(width), int(members), int(flags))


HOIST = {"single": 1, "double": 2}  # CKC_HOIST_SINGLE, CKC_HOIST_DOUBLE


def layer_create_conv(ctx: Context, layout: ckc_layout, out_ch, in_ch, ksize, stride, codebook, idx, bias,
                      level, pt_scale, bias_scale, stream=None, hoisting: str = "double") -> Layer:
    """hoisting: "double" (one ModDown per output) or "single" (one per
    rotated input); see ckc_layer_create_conv_ex."""
    if hoisting not in HOIST:
        raise ValueError(f"hoisting must be one of {sorted(HOIST)}, not {hoisting!r}")
    cb, cbp = _dbl(codebook)
    ix = np.ascontiguousarray(np.asarray(idx, dtype=np.uint16))
    if bias is not None:
        bb, bbp = _dbl(bias)
    else:
        bbp = None
    k = int(cb.shape[1])
    h = _vp()
    _check("ckc_layer_create_conv_ex", lib().ckc_layer_create_conv_ex(
        ctx.h, C.byref(layout), out_ch, in_ch, ksize, stride, k, cbp, ix.ctypes.data_as(C.POINTER(C.c_uint16)),
        bbp, level, float(pt_scale), float(bias_scale), HOIST[hoisting], C.byref(h), _stream(stream)))
    return Layer(ctx, h, "conv")


def layer_create_act(ctx: Context, layout: ckc_layout, channels, b, c, a_absorb, level, in_scale,
                     stream=None) -> Layer:
    bb, bbp = _dbl(b)
    cc, ccp = _dbl(c)
    h = _vp()
    _check("ckc_layer_create_act", lib().ckc_layer_create_act(ctx.h, C.byref(layout), channels, bbp, ccp,
                                                              float(a_absorb), level, float(in_scale), C.byref(h),
                                                              _stream(stream)))
    return Layer(ctx, h, "act")


def layer_create_dense(ctx: Context, layout: ckc_layout, classes, in_ch, w, bias, level, pt_scale, bias_scale,
                       stream=None) -> Layer:
    """w: [members][classes][in_ch] (after global average pooling) or
    [members][classes][in_ch][height][width] (over the flattened grid:
    ckc_layer_create_dense_spatial)."""
    ww, wp = _dbl(w)
    if bias is not None:
        bb, bbp = _dbl(bias)
    else:
        bbp = None
    h = _vp()
    fn = "ckc_layer_create_dense_spatial" if np.ndim(w) == 5 else "ckc_layer_create_dense"
    _check(fn, getattr(lib(), fn)(ctx.h, C.byref(layout), classes, in_ch, wp, bbp, level, float(pt_scale),
                                  float(bias_scale), C.byref(h), _stream(stream)))
    return Layer(ctx, h, "dense")


def _eval(fn, ctx, keys, layer, ins, n_img, outs, stream):
    ia, oa = _ct_array(ins), _ct_array(outs)
    _check(fn, getattr(lib(), fn)(ctx.h, keys.evk, layer.h, ia, n_img, oa, _stream(stream)))
    _update_all(outs, oa)
    return outs


def eval_conv(ctx, keys, layer, ins, n_img, outs, stream=None):
    return _eval("ckc_eval_conv", ctx, keys, layer, ins, n_img, outs, stream)


def eval_quad_act(ctx, keys, layer, ins, n_img, outs, stream=None):
    return _eval("ckc_eval_quad_act", ctx, keys, layer, ins, n_img, outs, stream)


def eval_dense(ctx, keys, layer, ins, n_img, outs, stream=None):
    return _eval("ckc_eval_dense", ctx, keys, layer, ins, n_img, outs, stream)


def eval_avgpool2(ctx, keys, layout: ckc_layout, ins, outs, stream=None):
    ia, oa = _ct_array(ins), _ct_array(outs)
    _check("ckc_eval_avgpool2", lib().ckc_eval_avgpool2(ctx.h, keys.evk, C.byref(layout), ia, len(ins), oa,
                                                        _stream(stream)))
    _update_all(outs, oa)
    return outs


def rescale_many(ctx, ins, outs, stream=None):
    ia, oa = _ct_array(ins), _ct_array(outs)
    _check("ckc_rescale_many", lib().ckc_rescale_many(ctx.h, ia, len(ins), oa, _stream(stream)))
    _update_all(outs, oa)
    return outs


def add_many(ctx, a, b, outs, stream=None):
    aa, ba, oa = _ct_array(a), _ct_array(b), _ct_array(outs)
    _check("ckc_add_many", lib().ckc_add_many(ctx.h, aa, ba, len(a), oa, _stream(stream)))
    _update_all(outs, oa)
    return outs


def rotate_many(ctx, keys, ins, steps, outs=None, stream=None):
    """outs[i * len(steps) + j] = Rot_{steps[j]}(ins[i]) (hoisted, batched)."""
    steps = list(steps)
    if outs is None:
        outs = [ctx.new_ct(c.level, 2, c.scale) for c in ins for _ in steps]
    ia, oa = _ct_array(ins), _ct_array(outs)
    st = (C.c_int32 * max(len(steps), 1))(*steps)
    _check("ckc_rotate_many", lib().ckc_rotate_many(ctx.h, keys.evk, ia, len(ins), st, len(steps), oa,
                                                    _stream(stream)))
    _update_all(outs, oa)
    return outs


def mul_relin_many(ctx, keys, a, b, outs=None, stream=None):
    """outs[i] = Relin(a[i] * b[i])."""
    if outs is None:
        outs = [ctx.new_ct(x.level, 2, x.scale) for x in a]
    aa, ba, oa = _ct_array(a), _ct_array(b), _ct_array(outs)
    _check("ckc_mul_relin_many", lib().ckc_mul_relin_many(ctx.h, keys.evk, aa, ba, len(a), oa, _stream(stream)))
    _update_all(outs, oa)
    return outs


def mac_plain_many(ctx, ins, pts, outs=None, stream=None):
    """outs[o] = sum_t ins[o * len(pts) + t] * pts[t]."""
    T = len(pts)
    n_out = len(ins) // T
    if outs is None:
        outs = [ctx.new_ct(ins[0].level, 2, ins[0].scale) for _ in range(n_out)]
    ia, oa = _ct_array(ins), _ct_array(outs)
    pa = (ckc_pt * T)(*[p.c() for p in pts])
    _check("ckc_mac_plain_many", lib().ckc_mac_plain_many(ctx.h, ia, pa, T, n_out, oa, _stream(stream)))
    _update_all(outs, oa)
    return outs


def prof_enable(on: bool = True):
    _check("ckc_prof_enable", lib().ckc_prof_enable(int(on)))


def prof_query(name: str) -> dict:
    n = C.c_int64()
    ms, by, wk = C.c_double(), C.c_double(), C.c_double()
    _check("ckc_prof_query", lib().ckc_prof_query(name.encode(), C.byref(n), C.byref(ms), C.byref(by), C.byref(wk)))
    return {"launches": int(n.value), "ms": ms.value, "bytes": by.value, "work": wk.value}


def variant_enable(on: bool = True):
    _check("ckc_variant_enable", lib().ckc_variant_enable(int(on)))


def variant_counts() -> dict:
    """Launches per kernel instantiation since variant_enable()."""
    buf = C.create_string_buffer(1 << 16)
    _check("ckc_variant_list", lib().ckc_variant_list(buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n = line.rsplit("=", 1)
        out[name] = int(n)
    return out


def tune_set(knob: str, value: int):
    _check("ckc_tune_set", lib().ckc_tune_set(knob.encode(), int(value)))


def tune_get(knob: str) -> int:
    v = C.c_int()
    _check("ckc_tune_get", lib().ckc_tune_get(knob.encode(), C.byref(v)))
    return int(v.value)


TUNE_KNOBS = {"conv_outs": (8, 16), "conv_imgs": (1, 2, 4), "ks_batch": (16, 32, 64), "conv_fuse": (1, 0),
              "conv_rows": (1, 2)}


def stream_release(stream=None):
    """Free the library's scratch arena of `stream` (after its queued work);
    the next call on the stream grows a new one."""
    _check("ckc_stream_release", lib().ckc_stream_release(_stream(stream)))


class Plan:
    """A network's layer program parsed by the native runner."""

    def __init__(self, ctx, program_json: str, layers: list):
        self.ctx, self.layers = ctx, list(layers)  # the handles must outlive the plan
        arr = (C.c_void_p * max(len(layers), 1))(*[l.h for l in layers])
        h = C.c_void_p()
        _check("ckc_batch_plan", lib().ckc_batch_plan(ctx.h, program_json.encode(), arr, len(layers), C.byref(h)))
        self.h = h
        v = [C.c_int() for _ in range(4)]
        _check("ckc_batch_plan_info", lib().ckc_batch_plan_info(self.h, *[C.byref(x) for x in v]))
        self.in_count, self.in_level, self.out_count, self.out_level = (int(x.value) for x in v)

    def run(self, evks: list, inputs: list, stream=None) -> list:
        """inputs[r]: request r's input ciphertexts; evks[r]: its KeyPair.
        Returns [r][out_count] output ciphertexts."""
        n = len(inputs)
        outs = [[self.ctx.new_ct(self.out_level) for _ in range(self.out_count)] for _ in range(n)]
        in_arrs = [_ct_array(row) for row in inputs]
        out_arrs = [_ct_array(row) for row in outs]
        pin = (C.c_void_p * max(n, 1))(*[C.cast(a, C.c_void_p) for a in in_arrs])
        pout = (C.c_void_p * max(n, 1))(*[C.cast(a, C.c_void_p) for a in out_arrs])
        pev = (C.c_void_p * max(n, 1))(*[k.evk for k in evks])
        _check("ckc_batch_run", lib().ckc_batch_run(self.h, pev, pin, n, pout, _stream(stream)))
        for row, a in zip(outs, out_arrs):
            _update_all(row, a)
        return outs

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ckc_batch_plan_destroy(self.h)
        except Exception:
            pass


def set_test_fault(call_index: int, code: int = -6):
    """Test-only: the call_index-th following layer evaluation call fails
    with `code` (CKC_EDEVICE by default); 0 disarms."""
    _check("ckc_set_test_fault", lib().ckc_set_test_fault(int(call_index), int(code)))


def stream_reserve(nbytes: int, stream=None):
    """Grow the library's scratch arena of `stream` to at least nbytes now."""
    _check("ckc_stream_reserve", lib().ckc_stream_reserve(_stream(stream), C.c_size_t(int(nbytes))))

PROF_KERNELS = ("ntt_fwd", "ntt_inv", "bconv", "kip", "moddown", "conv_contract", "act_tensor", "rescale",
                "dense_mac", "ew", "mac_plain", "tensor", "copy")
