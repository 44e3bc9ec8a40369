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
