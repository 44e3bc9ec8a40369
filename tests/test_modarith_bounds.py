"""Bounds the GPU modular arithmetic relies on, checked in exact integers on
the host: the Montgomery reduction of a carry-counted sum of NPROD products
(operands below q < 2^62, one of each pair times 2^64 mod q) lands below
(NPROD / 4 + 1) q, so ceil(NPROD / 4) conditional subtractions of q give the
residue; the sum fits the accumulator while NPROD is at most the
accumulator's product cap for q's bit length."""
import random

import pytest

from workloads.params import is_prime


def prime_below(bits):
    q = (1 << bits) - 1
    while not (q % (1 << 17) == 1 and is_prime(q)):
        q -= 1 if q % 2 == 0 else 2
    return q


def prod_cap(k):
    return (1 << (128 - 2 * k)) - 1 if k >= 61 else 64


@pytest.mark.parametrize("bits", [40, 50, 60, 61, 62])
def test_montgomery_reduction_of_accumulated_products(bits):
    q = prime_below(bits)
    inv = q
    for _ in range(5):
        inv = inv * (2 - q * inv) % 2 ** 64
    assert inv * q % 2 ** 64 == 1
    qinv = -inv % 2 ** 64
    R = 2 ** 64 % q
    rnd = random.Random(bits)
    for n in sorted({1, 2, 3, 5, 8, 9, 17, prod_cap(q.bit_length())} - {0}):
        if n > prod_cap(q.bit_length()):
            continue
        for trial in range(200):
            a = [q - 1] * n if trial == 0 else [rnd.randrange(q) for _ in range(n)]
            b = [q - 1] * n if trial == 0 else [rnd.randrange(q) for _ in range(n)]
            V = sum(x * (y * R % q) for x, y in zip(a, b))
            assert V < 2 ** 128
            lo, hi = V % 2 ** 64, V >> 64
            m = lo * qinv % 2 ** 64
            t = hi + (m * q >> 64) + (1 if lo else 0)
            assert t < (n / 4 + 1) * q and t < 2 ** 64
            for _ in range((n + 3) // 4):
                t = t - q if t >= q else t
            assert t == sum(x * y for x, y in zip(a, b)) % q
