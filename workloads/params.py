"""RNS-CKKS parameter sets with explicit prime chains.

The paper's framework picks its RNS moduli automatically from the requested
bit sizes (Appendix D, "Details on FHE Parameters"): the chain is ordered
q_0 (holds the output), q_1 .. q_L (dropped by rescaling, q_L first), then the
special primes P used to extend the modulus during key switching.

Moduli selection (paper-silent procedure, read from the printed chains of
Appendix D): every modulus is an NTT-friendly prime q = 2^b + k*2N + 1.  For a
run of primes of sizes b_1, b_2, ... the next prime is taken, among the nearest
unused candidate above 2^b and the nearest unused candidate below 2^b, as the
one that keeps sum(log2 q_i) - sum(b_i) closest to zero.  This greedy balance
reproduces, in order, the four main chains the paper prints for VGG-16,
ResNet-18, ResNet-20 and ResNet-32 (checked in tests/test_oracle_pins.py,
test_paper_chains_reproduced).

Every consumer takes the explicit lists below; nothing downstream re-derives
primes, so a change here changes both sides of a parity test alike.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from functools import lru_cache

# Deterministic Miller-Rabin bases: correct for every n < 3.3e24 (covers u64).
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _candidates(bits: int, two_n: int, above: bool):
    """NTT-friendly primes 2^bits + k*2N + 1, walking away from 2^bits."""
    k = 1 if above else -1
    step = 1 if above else -1
    while True:
        q = (1 << bits) + k * two_n + 1
        if q <= 2:
            return
        if is_prime(q):
            yield q
        k += step


def balanced_chain(sizes: list[int], two_n: int, exclude=()) -> list[int]:
    """Primes for the requested bit sizes, in chain order (greedy log balance)."""
    used = set(exclude)
    out: list[int] = []
    dev = 0.0  # sum(log2 q) - sum(bits) so far
    gens: dict[tuple[int, bool], object] = {}
    heads: dict[tuple[int, bool], int] = {}

    def head(bits, above):
        key = (bits, above)
        if key not in gens:
            gens[key] = _candidates(bits, two_n, above)
        while key not in heads or heads[key] in used:
            heads[key] = next(gens[key])
        return heads[key]

    for b in sizes:
        up, dn = head(b, True), head(b, False)
        d_up = dev + math.log2(up) - b
        d_dn = dev + math.log2(dn) - b
        q = up if abs(d_up) <= abs(d_dn) else dn
        dev = d_up if q == up else d_dn
        used.add(q)
        out.append(q)
    return out


def nearest_prime(bits: int, two_n: int, exclude=()) -> int:
    """Single NTT-friendly prime nearest 2^bits (ties: the one above)."""
    up = next(q for q in _candidates(bits, two_n, True) if q not in exclude)
    dn = next(q for q in _candidates(bits, two_n, False) if q not in exclude)
    return up if (up - (1 << bits)) <= ((1 << bits) - dn) else dn


@dataclass(frozen=True)
class ParamSet:
    name: str
    logN: int
    q: tuple            # q_0 .. q_L (q_0 holds the output, q_L is dropped first)
    p: tuple            # special primes for hybrid key switching
    alpha: int          # primes per key-switching digit (dnum = ceil((L+1)/alpha))
    delta_log2: float   # default encoding scale
    note: str = ""

    @property
    def N(self) -> int:
        return 1 << self.logN

    @property
    def L(self) -> int:
        return len(self.q) - 1

    def to_dict(self) -> dict:
        d = asdict(self)
        d["q"] = list(self.q)
        d["p"] = list(self.p)
        return d


@lru_cache(maxsize=None)
def tiny() -> ParamSet:
    """Small parity case: N=2^12, three 40-bit Q primes, one 50-bit P prime.

    Not a secure parameter set (log2 PQ = 170 at N = 2^12); it exists so the
    oracle can run the whole path in seconds.
    """
    two_n = 2 << 12
    q = balanced_chain([40, 40, 40], two_n)
    p = [nearest_prime(50, two_n, exclude=q)]
    return ParamSet("tiny", 12, tuple(q), tuple(p), alpha=1, delta_log2=40,
                    note="test-only, not secure")


@lru_cache(maxsize=None)
def mid() -> ParamSet:
    """Parity case for ring sizes other than 2^12 and 2^16 (the transforms'
    generic path): N=2^13, four 45-bit Q primes, two 50-bit P primes, two
    primes per digit."""
    two_n = 2 << 13
    q = balanced_chain([45] * 4, two_n)
    p = balanced_chain([50] * 2, two_n, exclude=q)
    return ParamSet("mid", 13, tuple(q), tuple(p), alpha=2, delta_log2=40,
                    note="test-only, not secure")


@lru_cache(maxsize=None)
def micro() -> ParamSet:
    """Kernel microbenchmark: N=2^16, 24 Q primes of 50 bits, 3 P primes of
    50 bits, three primes per digit (dnum = 8)."""
    two_n = 2 << 16
    q = balanced_chain([50] * 24, two_n)
    p = balanced_chain([50] * 3, two_n, exclude=q)
    return ParamSet("micro", 16, tuple(q), tuple(p), alpha=3, delta_log2=40,
                    note="log2 PQ ~ 1350")


@lru_cache(maxsize=None)
def resnet20_tower(levels: int = 20, big_bits: int = 60, delta_bits: int = 30,
                   p_bits: int = 61, n_p: int = 3, alpha: int = 3) -> ParamSet:
    """ResNet-20-style chain with tower reuse (Section 4.3): q_i ~ Delta^2.

    q_0 .. q_{L-1} are big_bits-bit primes (q_0 holds the output), q_L ~ Delta
    is the prime the first convolution is rescaled by.  L = 20 as the paper
    reports for ResNet-20 with all structural optimisations.
    """
    two_n = 2 << 16
    q = balanced_chain([big_bits] * levels, two_n)
    q.append(nearest_prime(delta_bits, two_n, exclude=q))
    p = balanced_chain([p_bits] * n_p, two_n, exclude=q)
    return ParamSet(f"resnet20_tower_L{levels}", 16, tuple(q), tuple(p),
                    alpha=alpha, delta_log2=delta_bits,
                    note="tower reuse, q_i ~ Delta^2")


@lru_cache(maxsize=None)
def small_tower(logN: int = 12, levels: int = 4, big_bits: int = 60,
                delta_bits: int = 30, p_bits: int = 61, n_p: int = 2,
                alpha: int = 2) -> ParamSet:
    """Reduced-ring variant of the tower chain for network-level parity runs."""
    two_n = 2 << logN
    q = balanced_chain([big_bits] * levels, two_n)
    q.append(nearest_prime(delta_bits, two_n, exclude=q))
    p = balanced_chain([p_bits] * n_p, two_n, exclude=q)
    return ParamSet(f"small_tower_N{logN}_L{levels}", logN, tuple(q), tuple(p),
                    alpha=alpha, delta_log2=delta_bits, note="test-only")


@lru_cache(maxsize=None)
def chw_chain(logN: int = 12, levels: int = 4, delta_bits: int = 40) -> ParamSet:
    """A plain (non-tower) chain for the CHW-layout network: a 60-bit q_0 that
    holds the logits, `levels` primes of delta_bits bits that the rescales
    drop (one per layer), one 61-bit special prime, one prime per digit.
    Test and measurement only."""
    two_n = 2 << logN
    q0 = nearest_prime(60, two_n)
    q = [q0] + balanced_chain([delta_bits] * levels, two_n, exclude=[q0])
    p = [nearest_prime(61, two_n, exclude=q)]
    return ParamSet(f"chw_N{logN}_L{levels}", logN, tuple(q), tuple(p), alpha=1, delta_log2=delta_bits,
                    note="test-only")


def by_name(name: str) -> ParamSet:
    table = {"tiny": tiny, "mid": mid, "micro": micro}
    if name in table:
        return table[name]()
    raise KeyError(name)
