"""Bounds the GPU modular arithmetic relies on, checked in exact integers on
the host against a host build of the library's own reduction
(paper_2509_22857_amd/csrc/modarith.h, compiled host-only with hipcc): the
Montgomery reduction of a carry-counted sum of NPROD products (operands
below q < 2^62) must return value * 2^-64 mod q for every value below
NPROD q^2 -- including the worst case, where m = lo * qinv mod 2^64 is close
to 2^64 and hi is at its largest, in which the unreduced quotient
hi + mulhi(m, q) + 1 exceeds 2^64 for q near 2^62 and NPROD >= 12 -- and the
sum must fit the accumulator while NPROD is at most the accumulator's
product cap for q's bit length."""
import ctypes
import os
import random
import shutil
import subprocess

import pytest

from workloads.params import is_prime

HERE = os.path.dirname(os.path.abspath(__file__))
SHIM_NPROD = list(range(1, 18)) + [64, 65]


def prime_below(bits):
    q = (1 << bits) - 1
    while not (q % (1 << 17) == 1 and is_prime(q)):
        q -= 1 if q % 2 == 0 else 2
    return q


def prod_cap(k):
    return (1 << (128 - 2 * k)) - 1 if k >= 61 else 64


def qinv_of(q):
    inv = q
    for _ in range(6):
        inv = inv * (2 - q * inv) % 2 ** 64
    assert inv * q % 2 ** 64 == 1
    return -inv % 2 ** 64


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("modarith") / "shim.so"
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O2", "-fPIC", "-shared",
                    os.path.join(HERE, "modarith_shim.cpp"), "-o", str(out)], check=True)
    lib = ctypes.CDLL(str(out))
    lib.shim_redc.restype = ctypes.c_uint64
    lib.shim_redc.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    return lib


def worst_sums(q, n, count=4):
    """Sums of n products of residues whose low word makes m = lo * qinv mod
    2^64 equal (or close to) 2^64 - 1 while hi stays near its maximum: n - 1
    products (q - 1)^2 and a last product x w with x w = q - rest mod 2^64
    (then lo = q, m = 2^64 - 1), for odd w just below q and x < q."""
    rest = (n - 1) * (q - 1) ** 2
    out = []
    w = q - 2
    while len(out) < count and w > q - 2 * 10 ** 5:
        for target in (q, 2 * q, 3 * q):
            x = (target - rest) * pow(w, -1, 2 ** 64) % 2 ** 64
            if x < q:
                out.append(rest + x * w)
        w -= 2
    return out


@pytest.mark.parametrize("bits", [40, 50, 60, 61, 62])
def test_montgomery_reduction_of_accumulated_products(bits, shim):
    q = prime_below(bits)
    qinv = qinv_of(q)
    R = 2 ** 64 % q
    Rinv = pow(R, -1, q)
    rnd = random.Random(bits)
    cap = prod_cap(q.bit_length())
    for n in [n for n in SHIM_NPROD if n <= cap]:
        # below 50 bits a product x w < q^2 rarely has the required low word
        cases = worst_sums(q, n) if bits >= 50 else []
        assert cases or bits < 50, (bits, n)
        cases.append(n * (q - 1) ** 2)
        for _ in range(100):
            cases.append(sum(rnd.randrange(q) * rnd.randrange(q) for _ in range(n)))
        for V in cases:
            assert V < n * q * q and V < 2 ** 128
            hi, lo = V >> 64, V % 2 ** 64
            got = shim.shim_redc(n, hi, lo, q, qinv)
            assert got == V * Rinv % q, (bits, n, hex(V))


def test_worst_case_quotient_exceeds_64_bits_near_2_62():
    """The case the reduction guards against: without first reducing hi, the
    quotient of a worst-case sum of 13..15 products wraps at q ~ 2^62."""
    q = 0x3fffffffffe80001
    assert is_prime(q)
    qinv = qinv_of(q)
    for n in (13, 14, 15):
        V = max(worst_sums(q, n))
        hi, lo = V >> 64, V % 2 ** 64
        m = lo * qinv % 2 ** 64
        assert hi + (m * q >> 64) + 1 >= 2 ** 64, n


def _shim_fold(shim):
    shim.shim_fold_cap.restype = ctypes.c_int
    shim.shim_fold_cap.argtypes = [ctypes.c_int]
    shim.shim_accc_value.restype = None
    shim.shim_accc_value.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(ctypes.c_uint64)]


class _Acc:
    """The carry-counted accumulator of modarith.h as exact integers: every
    64-bit word and 32-bit counter is checked not to wrap where the device
    code relies on it (h has no carry counter; l and m count theirs)."""

    def __init__(self, l=0):
        self.h = self.m = self.cm = self.cl = 0
        self.l = l

    def macc(self, a, b):
        a0, a1, b0, b1 = a & 0xFFFFFFFF, a >> 32, b & 0xFFFFFFFF, b >> 32
        self.l += a0 * b0
        self.cl += self.l >> 64
        self.l &= 2 ** 64 - 1
        for t in (a0 * b1, a1 * b0):
            self.m += t
            self.cm += self.m >> 64
            self.m &= 2 ** 64 - 1
        self.h += a1 * b1
        assert self.h < 2 ** 64, "h wrapped"
        assert self.cl < 2 ** 32 and self.cm < 2 ** 32

    def exact(self):
        return self.l + (self.cl << 64) + (self.m << 32) + (self.cm << 96) + (self.h << 64)


@pytest.mark.parametrize("bits", [30, 50, 60, 61, 62])
def test_folded_accumulator_holds_long_sums(bits, shim):
    """A long sum (a 512-input 3x3 contraction: 4608 products) accumulated
    with a fold whenever fold_cap(k) products have gone in since the last
    one: with operands at q - 1 (the largest h growth) and at random, h never
    wraps, the library's accc_value never wraps, and the result is the sum
    mod q."""
    _shim_fold(shim)
    q = prime_below(bits)
    k = q.bit_length()
    cap = shim.shim_fold_cap(k)
    assert cap >= 3
    r64 = 2 ** 64 % q
    rnd = random.Random(bits)
    hi, lo = ctypes.c_uint64(), ctypes.c_uint64()

    def value(acc):
        shim.shim_accc_value(acc.h, acc.m, acc.l, acc.cm, acc.cl, ctypes.byref(hi), ctypes.byref(lo))
        v = (hi.value << 64) | lo.value
        assert v == acc.exact(), "accc_value wrapped"
        return v

    for kind in ("max", "random"):
        acc, cnt, want = _Acc(), 0, 0
        for _ in range(4608):
            if cnt == cap:
                v = value(acc)
                acc = _Acc(v & (2 ** 64 - 1))
                acc.macc(v >> 64, r64)
                cnt = 0
            a, b = (q - 1, q - 1) if kind == "max" else (rnd.randrange(q), rnd.randrange(q))
            acc.macc(a, b)
            want += a * b
            cnt += 1
        assert value(acc) % q == want % q

