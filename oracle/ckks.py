"""Python face of the CPU oracle (RNS-CKKS over the plain C core).

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The product path never does.

Every ciphertext here is held in coefficient form as a numpy uint64 array of
shape [npoly][level+1][N] (limb l is reduced modulo q_l), with its level and
its scale (a double).  The operations follow the RNS-CKKS description of the
paper's Section 2.2 ("Leveled Fully Homomorphic Encryption") under the
canonical readings recorded in the design notes (key-switching digits, the
order of automorphism and ModUp, rounding in rescale, the encoding FFT).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_u64p = C.POINTER(C.c_uint64)
_dblp = C.POINTER(C.c_double)
_i8p = C.POINTER(C.c_int8)

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.oc_create.restype = C.c_void_p
        L.oc_create.argtypes = [C.c_int, C.c_int, _u64p, C.c_int, _u64p]
        L.oc_destroy.argtypes = [C.c_void_p]
        L.oc_psi.restype = C.c_uint64
        L.oc_psi.argtypes = [C.c_void_p, C.c_int]
        for name in ("oc_ntt", "oc_intt"):
            getattr(L, name).argtypes = [C.c_void_p, C.c_int, _u64p]
        L.oc_polymul.argtypes = [C.c_void_p, C.c_int, _u64p, _u64p, _u64p]
        L.oc_automorphism.argtypes = [C.c_void_p, C.c_int, _u64p, C.c_uint64, _u64p]
        L.oc_galois_elt.restype = C.c_uint64
        L.oc_galois_elt.argtypes = [C.c_void_p, C.c_int64]
        L.oc_stream_key.restype = C.c_uint64
        L.oc_stream_key.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.oc_draw.restype = C.c_uint64
        L.oc_draw.argtypes = [C.c_uint64, C.c_uint64]
        L.oc_sample_secret.argtypes = [C.c_void_p, C.c_uint64, _i8p]
        L.oc_keygen_switch.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_int, _i8p, _u64p, _u64p]
        L.oc_encrypt.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, _i8p, _u64p, C.c_int, _u64p]
        L.oc_decrypt.argtypes = [C.c_void_p, _i8p, _u64p, C.c_int, C.c_int, _u64p]
        L.oc_modup_digit.argtypes = [C.c_void_p, _u64p, C.c_int, C.c_int, C.c_int, _u64p]
        L.oc_moddown.argtypes = [C.c_void_p, _u64p, C.c_int, _u64p]
        L.oc_keyswitch.argtypes = [C.c_void_p, _u64p, C.c_int, C.c_int, C.c_uint64, _u64p, _u64p]
        L.oc_keyswitch_ext.argtypes = [C.c_void_p, _u64p, C.c_int, C.c_int, C.c_uint64, _u64p, _u64p]
        L.oc_encode_ext.argtypes = [C.c_void_p, _dblp, _dblp, C.c_size_t, C.c_double, C.c_int, _u64p]
        L.oc_rescale.argtypes = [C.c_void_p, _u64p, C.c_int, C.c_int, _u64p]
        L.oc_encode.argtypes = [C.c_void_p, _dblp, _dblp, C.c_size_t, C.c_double, C.c_int, _u64p, _dblp]
        L.oc_decode.argtypes = [C.c_void_p, _dblp, C.c_double, _dblp, _dblp]
        L.oc_const_residues.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, _u64p]
        _lib = L
    return _lib


def _p(a: np.ndarray, typ=_u64p):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(typ)


@dataclass
class Ct:
    """Ciphertext in coefficient form: data[npoly][level+1][N]."""
    data: np.ndarray
    level: int
    scale: float

    @property
    def npoly(self) -> int:
        return self.data.shape[0]

    def copy(self) -> "Ct":
        return Ct(self.data.copy(), self.level, self.scale)


@dataclass
class Pt:
    """Plaintext in coefficient form: data[level+1][N]."""
    data: np.ndarray
    level: int
    scale: float


@dataclass
class SecretKey:
    seed: int
    s: np.ndarray  # int8 ternary coefficients


class Oracle:
    """RNS-CKKS context over an explicit prime list (q_0..q_L then P)."""

    def __init__(self, logN: int, q, p, alpha: int):
        self.logN = int(logN)
        self.N = 1 << self.logN
        self.q = [int(x) for x in q]
        self.p = [int(x) for x in p]
        self.alpha = int(alpha)
        self.nq, self.np_ = len(self.q), len(self.p)
        self.L = self.nq - 1
        self.mod = self.q + self.p
        qa = np.array(self.q, dtype=np.uint64)
        pa = np.array(self.p, dtype=np.uint64)
        self._h = lib().oc_create(self.logN, self.nq, _p(qa), self.np_, _p(pa))
        if not self._h:
            raise ValueError("oracle context creation failed")
        self.dnum = (self.nq + self.alpha - 1) // self.alpha

    @classmethod
    def from_params(cls, ps) -> "Oracle":
        return cls(ps.logN, ps.q, ps.p, ps.alpha)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oc_destroy(h)
            self._h = None

    # ----------------------------------------------------------- limb level
    def prime_index(self, level: int, tt: int) -> int:
        """Target index tt of an extended basis at `level` -> prime index."""
        return tt if tt <= level else self.nq + (tt - level - 1)

    def ntt(self, a: np.ndarray, t: int) -> np.ndarray:
        x = np.ascontiguousarray(a, dtype=np.uint64).copy()
        lib().oc_ntt(self._h, t, _p(x))
        return x

    def intt(self, a: np.ndarray, t: int) -> np.ndarray:
        x = np.ascontiguousarray(a, dtype=np.uint64).copy()
        lib().oc_intt(self._h, t, _p(x))
        return x

    def polymul(self, a: np.ndarray, b: np.ndarray, t: int) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        o = np.empty(self.N, dtype=np.uint64)
        lib().oc_polymul(self._h, t, _p(a), _p(b), _p(o))
        return o

    def automorphism(self, a: np.ndarray, g: int, t: int) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64)
        o = np.empty(self.N, dtype=np.uint64)
        lib().oc_automorphism(self._h, t, _p(a), g, _p(o))
        return o

    def galois_elt(self, r: int) -> int:
        return int(lib().oc_galois_elt(self._h, int(r)))

    def psi(self, t: int) -> int:
        return int(lib().oc_psi(self._h, t))

    # ------------------------------------------------------------ keys
    def secret_key(self, seed: int) -> SecretKey:
        s = np.empty(self.N, dtype=np.int8)
        lib().oc_sample_secret(self._h, seed, _p(s, _i8p))
        return SecretKey(int(seed), s)

    def secret_limbs(self, sk: SecretKey) -> np.ndarray:
        """s reduced modulo every prime: [nprimes][N]."""
        s64 = sk.s.astype(np.int64)
        return np.stack([(s64 % m).astype(np.uint64) for m in self.mod])

    def switch_key(self, sk: SecretKey, key_id: int, sprime: np.ndarray) -> np.ndarray:
        """Hybrid key-switching key from s' (limbs over every prime) to s."""
        sprime = np.ascontiguousarray(sprime, dtype=np.uint64)
        assert sprime.shape == (len(self.mod), self.N)
        key = np.empty((self.dnum, 2, len(self.mod), self.N), dtype=np.uint64)
        lib().oc_keygen_switch(self._h, sk.seed, key_id, self.alpha, _p(sk.s, _i8p), _p(sprime), _p(key))
        return key

    def relin_key(self, sk: SecretKey) -> np.ndarray:
        sl = self.secret_limbs(sk)
        s2 = np.stack([self.polymul(sl[t], sl[t], t) for t in range(len(self.mod))])
        return self.switch_key(sk, 0, s2)

    def galois_key(self, sk: SecretKey, g: int) -> np.ndarray:
        sl = self.secret_limbs(sk)
        sg = np.stack([self.automorphism(sl[t], g, t) for t in range(len(self.mod))])
        return self.switch_key(sk, g, sg)

    # ------------------------------------------------------------ encoding
    def encode(self, z, level: int, scale: float) -> Pt:
        z = np.asarray(z)
        zr = np.ascontiguousarray(np.real(z), dtype=np.float64)
        zi = np.ascontiguousarray(np.imag(z), dtype=np.float64) if np.iscomplexobj(z) else None
        m = np.empty((level + 1, self.N), dtype=np.uint64)
        lib().oc_encode(self._h, _p(zr, _dblp), _p(zi, _dblp) if zi is not None else None,
                        len(zr), float(scale), level, _p(m), None)
        return Pt(m, level, float(scale))

    def encode_w(self, z) -> np.ndarray:
        """The unrounded encoding vector w (before scaling), for tests."""
        z = np.asarray(z)
        zr = np.ascontiguousarray(np.real(z), dtype=np.float64)
        zi = np.ascontiguousarray(np.imag(z), dtype=np.float64) if np.iscomplexobj(z) else None
        m = np.empty((1, self.N), dtype=np.uint64)
        w = np.empty(self.N, dtype=np.float64)
        lib().oc_encode(self._h, _p(zr, _dblp), _p(zi, _dblp) if zi is not None else None,
                        len(zr), 1.0, 0, _p(m), _p(w, _dblp))
        return w

    def const_residues(self, value: float, scale: float, nl: int) -> np.ndarray:
        out = np.empty(nl, dtype=np.uint64)
        lib().oc_const_residues(self._h, float(value), float(scale), nl, _p(out))
        return out

    def lift_q0(self, m0: np.ndarray) -> np.ndarray:
        """Centred lift of a q_0 limb to signed integers (as Python-exact int64)."""
        q0 = self.q[0]
        v = m0.astype(np.int64, copy=True) if q0 < (1 << 63) else None
        half = q0 >> 1
        v = np.where(m0 > half, m0.astype(np.int64) - np.int64(q0), m0.astype(np.int64))
        return v

    def decode(self, m: np.ndarray, scale: float, complex_out: bool = False):
        """Decode from a coefficient-form plaintext (only limb 0 is used)."""
        m0 = np.asarray(m)[0] if np.asarray(m).ndim == 2 else np.asarray(m)
        coef = np.ascontiguousarray(self.lift_q0(m0).astype(np.float64))
        n = self.N // 2
        zr = np.empty(n)
        zi = np.empty(n)
        lib().oc_decode(self._h, _p(coef, _dblp), float(scale), _p(zr, _dblp), _p(zi, _dblp))
        return zr + 1j * zi if complex_out else zr

    # ---------------------------------------------------- encrypt / decrypt
    def encrypt(self, pt: Pt, sk: SecretKey, stream_id: int) -> Ct:
        m = np.ascontiguousarray(pt.data, dtype=np.uint64)
        ct = np.empty((2, pt.level + 1, self.N), dtype=np.uint64)
        lib().oc_encrypt(self._h, sk.seed, stream_id, _p(sk.s, _i8p), _p(m), pt.level, _p(ct))
        return Ct(ct, pt.level, pt.scale)

    def decrypt(self, ct: Ct, sk: SecretKey) -> np.ndarray:
        d = np.ascontiguousarray(ct.data, dtype=np.uint64)
        m = np.empty((ct.level + 1, self.N), dtype=np.uint64)
        lib().oc_decrypt(self._h, _p(sk.s, _i8p), _p(d), ct.npoly, ct.level, _p(m))
        return m

    def decrypt_decode(self, ct: Ct, sk: SecretKey, complex_out: bool = False):
        return self.decode(self.decrypt(ct, sk), ct.scale, complex_out)

    # ------------------------------------------------------- key switching
    def modup_digit(self, d: np.ndarray, level: int, j: int) -> np.ndarray:
        d = np.ascontiguousarray(d, dtype=np.uint64)
        out = np.empty((level + 1 + self.np_, self.N), dtype=np.uint64)
        lib().oc_modup_digit(self._h, _p(d), level, self.alpha, j, _p(out))
        return out

    def moddown(self, x: np.ndarray, level: int) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty((level + 1, self.N), dtype=np.uint64)
        lib().oc_moddown(self._h, _p(x), level, _p(out))
        return out

    def keyswitch_ext(self, d: np.ndarray, level: int, key: np.ndarray, g: int = 1) -> np.ndarray:
        """The key switch before ModDown: [2][level+1+np][N] over Q_l then P."""
        d = np.ascontiguousarray(d, dtype=np.uint64)
        key = np.ascontiguousarray(key, dtype=np.uint64)
        acc = np.empty((2, level + 1 + len(self.p), self.N), dtype=np.uint64)
        lib().oc_keyswitch_ext(self._h, _p(d), level, self.alpha, g, _p(key), _p(acc))
        return acc

    def encode_ext(self, z, level: int, scale: float) -> np.ndarray:
        """The encoding of z reduced into q_0..q_level and every P prime:
        [level+1+np][N] coefficient form."""
        z = np.asarray(z)
        zr = np.ascontiguousarray(np.real(z), dtype=np.float64)
        zi = np.ascontiguousarray(np.imag(z), dtype=np.float64) if np.iscomplexobj(z) else None
        m = np.empty((level + 1 + len(self.p), self.N), dtype=np.uint64)
        lib().oc_encode_ext(self._h, _p(zr, _dblp), _p(zi, _dblp) if zi is not None else None,
                            len(zr), float(scale), level, _p(m))
        return m

    def keyswitch(self, d: np.ndarray, level: int, key: np.ndarray, g: int = 1) -> np.ndarray:
        d = np.ascontiguousarray(d, dtype=np.uint64)
        key = np.ascontiguousarray(key, dtype=np.uint64)
        u = np.empty((2, level + 1, self.N), dtype=np.uint64)
        lib().oc_keyswitch(self._h, _p(d), level, self.alpha, g, _p(key), _p(u))
        return u

    # ------------------------------------------------------ homomorphic ops
    def _limbwise(self, a: np.ndarray, b: np.ndarray, op) -> np.ndarray:
        """Apply op limb-wise modulo q_l with Python-int-free uint64 math."""
        out = np.empty_like(a)
        nl = a.shape[-2]
        for l in range(nl):
            q = np.uint64(self.q[l])
            out[..., l, :] = op(a[..., l, :], b[..., l, :], q)
        return out

    @staticmethod
    def _add(a, b, q):
        s = a + b  # q < 2^62: no wrap
        return np.where(s >= q, s - q, s)

    @staticmethod
    def _sub(a, b, q):
        return np.where(a >= b, a - b, a + (q - b))

    def add(self, a: Ct, b: Ct) -> Ct:
        self._check_pair(a, b)
        npoly = max(a.npoly, b.npoly)
        out = np.zeros((npoly, a.level + 1, self.N), dtype=np.uint64)
        out[:a.npoly] = a.data
        out[:b.npoly] = self._limbwise(out[:b.npoly], b.data, self._add)
        return Ct(out, a.level, a.scale)

    def sub(self, a: Ct, b: Ct) -> Ct:
        self._check_pair(a, b)
        npoly = max(a.npoly, b.npoly)
        out = np.zeros((npoly, a.level + 1, self.N), dtype=np.uint64)
        out[:a.npoly] = a.data
        out[:b.npoly] = self._limbwise(out[:b.npoly], b.data, self._sub)
        return Ct(out, a.level, a.scale)

    def _check_pair(self, a: Ct, b: Ct):
        if a.level != b.level:
            raise ValueError("level mismatch")
        if abs(a.scale / b.scale - 1.0) > 2.0 ** -30:
            raise ValueError("scale mismatch")

    def add_plain(self, a: Ct, p: Pt) -> Ct:
        if p.level < a.level:
            raise ValueError("plaintext level too low")
        if abs(a.scale / p.scale - 1.0) > 2.0 ** -30:
            raise ValueError("scale mismatch")
        out = a.data.copy()
        out[0] = self._limbwise(out[0][None], p.data[None, :a.level + 1], self._add)[0]
        return Ct(out, a.level, a.scale)

    def add_const(self, a: Ct, value: float) -> Ct:
        """Add value*scale (rounded) to every slot: coefficient 0 of c0."""
        r = self.const_residues(value, a.scale, a.level + 1)
        out = a.data.copy()
        for l in range(a.level + 1):
            q = self.q[l]
            out[0, l, 0] = np.uint64((int(out[0, l, 0]) + int(r[l])) % q)
        return Ct(out, a.level, a.scale)

    def mul_const(self, a: Ct, value: float, scale: float) -> Ct:
        """Multiply by the constant round(value * scale) (the encoding of the
        all-`value` slot vector, Section 2.2): every limb times its residue."""
        r = self.const_residues(value, scale, a.level + 1)
        out = np.empty_like(a.data)
        for k in range(a.npoly):
            for l in range(a.level + 1):
                q = self.q[l]
                out[k, l] = ((a.data[k, l].astype(object) * int(r[l])) % q).astype(np.uint64)
        return Ct(out, a.level, a.scale * scale)

    def mul_plain(self, a: Ct, p: Pt) -> Ct:
        if p.level < a.level:
            raise ValueError("plaintext level too low")
        out = np.empty_like(a.data)
        for k in range(a.npoly):
            for l in range(a.level + 1):
                out[k, l] = self.polymul(a.data[k, l], p.data[l], l)
        return Ct(out, a.level, a.scale * p.scale)

    def tensor(self, a: Ct, b: Ct) -> Ct:
        """(a0,a1) x (b0,b1) -> (a0 b0, a0 b1 + a1 b0, a1 b1)."""
        if a.level != b.level or a.npoly != 2 or b.npoly != 2:
            raise ValueError("tensor needs two 2-poly ciphertexts at one level")
        nl = a.level + 1
        out = np.empty((3, nl, self.N), dtype=np.uint64)
        for l in range(nl):
            q = np.uint64(self.q[l])
            a0b0 = self.polymul(a.data[0, l], b.data[0, l], l)
            a0b1 = self.polymul(a.data[0, l], b.data[1, l], l)
            a1b0 = self.polymul(a.data[1, l], b.data[0, l], l)
            a1b1 = self.polymul(a.data[1, l], b.data[1, l], l)
            out[0, l] = a0b0
            out[1, l] = self._add(a0b1, a1b0, q)
            out[2, l] = a1b1
        return Ct(out, a.level, a.scale * b.scale)

    def relin(self, a: Ct, rlk: np.ndarray) -> Ct:
        if a.npoly != 3:
            raise ValueError("relinearisation needs a 3-poly ciphertext")
        u = self.keyswitch(a.data[2], a.level, rlk, 1)
        out = np.empty((2, a.level + 1, self.N), dtype=np.uint64)
        out[0] = self._limbwise(a.data[0][None], u[0][None], self._add)[0]
        out[1] = self._limbwise(a.data[1][None], u[1][None], self._add)[0]
        return Ct(out, a.level, a.scale)

    def rotate(self, a: Ct, r: int, gkey: np.ndarray | None) -> Ct:
        """Left rotation of the slots by r: (sigma_g c0 + u0, u1) with
        u = ModDown(sum_j sigma_g(ModUp_j(c1)) * key_g,j); r = 0 is identity."""
        if a.npoly != 2:
            raise ValueError("rotation needs a 2-poly ciphertext")
        g = self.galois_elt(r)
        if g == 1:
            return a.copy()
        u = self.keyswitch(a.data[1], a.level, gkey, g)
        nl = a.level + 1
        out = np.empty((2, nl, self.N), dtype=np.uint64)
        for l in range(nl):
            q = np.uint64(self.q[l])
            out[0, l] = self._add(self.automorphism(a.data[0, l], g, l), u[0, l], q)
            out[1, l] = u[1, l]
        return Ct(out, a.level, a.scale)

    def rescale(self, a: Ct) -> Ct:
        if a.level < 1:
            raise ValueError("cannot rescale at level 0")
        d = np.ascontiguousarray(a.data, dtype=np.uint64)
        out = np.empty((a.npoly, a.level, self.N), dtype=np.uint64)
        lib().oc_rescale(self._h, _p(d), a.npoly, a.level, _p(out))
        return Ct(out, a.level - 1, a.scale / float(self.q[a.level]))

    def mod_drop(self, a: Ct, to_level: int) -> Ct:
        if to_level > a.level or to_level < 0:
            raise ValueError("bad target level")
        return Ct(np.ascontiguousarray(a.data[:, :to_level + 1]), to_level, a.scale)
