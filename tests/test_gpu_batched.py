"""GPU <-> oracle parity of the batched entry points (rotate_many,
mul_relin_many, mac_plain_many), through the C-ABI.

The batched forms share one ModUp per input across rotation steps and read
each key or plaintext once per launch; every output is compared bit-exactly
(coefficient form) with the oracle applied to that ciphertext alone.  The
parameter sets cover every digit count the key inner product specialises
(1..8) and the generic path (more than 8 digits), and batches above the
64-ciphertext launch limit.
"""
import numpy as np
import pytest

from workloads import gen
from workloads.params import ParamSet, balanced_chain, tiny, mid, micro

pytestmark = pytest.mark.gpu


def wide_digits() -> ParamSet:
    """N = 2^12, 10 primes of 40 bits, one digit per prime (dnum = 10)."""
    q = balanced_chain([40] * 10, 2 << 12)
    p = balanced_chain([50], 2 << 12, exclude=q)
    return ParamSet("wide_digits", 12, tuple(q), tuple(p), alpha=1, delta_log2=40, note="test-only")


def _setup(ps):
    import torch
    from paper_2509_22857_amd.ckks import Context
    from oracle.ckks import Oracle
    print(f"[batched] params={ps.name} N={ps.N} nq={len(ps.q)} np={len(ps.p)} alpha={ps.alpha}", flush=True)
    return Context.from_params(ps), Oracle.from_params(ps), torch


def _cts(ctx, ps, seeds, level, scale=1.0):
    raw = [gen.random_ct(s, ps.q, level, ps.N) for s in seeds]
    return raw, [ctx.ct_from_coeff(a, level, scale) for a in raw]


@pytest.mark.parametrize("which,level,n,steps", [
    ("tiny", 2, 67, [0, 1, -1, 31]),     # 67 inputs: two launches, the second with 3
    ("wide", 9, 3, [1, -4]),             # dnum 10: generic digit loop
    ("micro", 23, 3, [-33, 0, 1]),       # dnum 8 at the top level
    ("micro", 19, 2, [1]),               # dnum 7
    ("mid", 3, 3, [1, -2, 0]),           # N = 2^13: the transforms' generic path
])
def test_rotate_many_bit_exact(which, level, n, steps):
    from oracle.ckks import Ct
    from paper_2509_22857_amd import ckks
    ps = {"tiny": tiny, "wide": wide_digits, "micro": micro, "mid": mid}[which]()
    ctx, orc, torch = _setup(ps)
    seed = 31
    keys = ctx.keygen(seed, [s for s in steps if s])
    sk = orc.secret_key(seed)
    raw, cts = _cts(ctx, ps, range(100, 100 + n), level)
    outs = ckks.rotate_many(ctx, keys, cts, steps)
    assert len(outs) == n * len(steps)
    # oracle on a sample of (input, step) pairs: first and last inputs, every step
    check_inputs = sorted({0, n - 1}) if which == "micro" else range(n)
    gks = {}
    for i in check_inputs:
        for j, r in enumerate(steps):
            if which == "micro" and i == 0 and j > 0 and r != 0:
                continue
            g = orc.galois_elt(r)
            if g != 1 and g not in gks:
                gks[g] = orc.galois_key(sk, g)
            want = orc.rotate(Ct(raw[i], level, 1.0), r, gks.get(g))
            got = outs[i * len(steps) + j]
            assert got.level == level and got.npoly == 2
            assert np.array_equal(ctx.ct_to_coeff(got), want.data), (i, r)


@pytest.mark.parametrize("which,level,n", [("tiny", 2, 66), ("wide", 6, 2), ("micro", 23, 2), ("mid", 2, 3)])
def test_mul_relin_many_bit_exact(which, level, n):
    from oracle.ckks import Ct
    from paper_2509_22857_amd import ckks
    ps = {"tiny": tiny, "wide": wide_digits, "micro": micro, "mid": mid}[which]()
    ctx, orc, torch = _setup(ps)
    seed = 77
    keys = ctx.keygen(seed, [])
    rlk = orc.relin_key(orc.secret_key(seed))
    ra, a = _cts(ctx, ps, range(200, 200 + n), level, 2.0 ** 20)
    rb, b = _cts(ctx, ps, range(400, 400 + n), level, 2.0 ** 21)
    # a != b for even i, squaring (b = a) for odd i
    bb = [a[i] if i % 2 else b[i] for i in range(n)]
    rbb = [ra[i] if i % 2 else rb[i] for i in range(n)]
    outs = ckks.mul_relin_many(ctx, keys, a, bb)
    check = range(n) if which != "micro" else (0, n - 1)
    for i in check:
        x, y = Ct(ra[i], level, 2.0 ** 20), Ct(rbb[i], level, bb[i].scale)
        want = orc.relin(orc.tensor(x, y), rlk)
        assert outs[i].scale == x.scale * y.scale
        assert np.array_equal(ctx.ct_to_coeff(outs[i]), want.data), i


@pytest.mark.parametrize("which,level,n_out,T", [("tiny", 2, 9, 7), ("tiny", 1, 2, 64), ("micro", 23, 2, 9)])
def test_mac_plain_many_bit_exact(which, level, n_out, T):
    from oracle.ckks import Ct, Pt
    from paper_2509_22857_amd import ckks
    ps = {"tiny": tiny, "micro": micro}[which]()
    ctx, orc, torch = _setup(ps)
    raw, cts = _cts(ctx, ps, range(600, 600 + n_out * T), level, 2.0 ** 30)
    # plaintexts one level above the ciphertexts where possible (extra limbs ignored)
    plev = min(level + 1, len(ps.q) - 1)
    praw = [gen.random_limbs(900 + t, ps.q[:plev + 1], ps.N) for t in range(T)]
    pts = [ctx.pt_from_coeff(p, plev, 2.0 ** 25) for p in praw]
    outs = ckks.mac_plain_many(ctx, cts, pts)
    assert len(outs) == n_out
    for o in ((0, n_out - 1) if which == "micro" else range(n_out)):
        acc = None
        for t in range(T):
            term = orc.mul_plain(Ct(raw[o * T + t], level, 2.0 ** 30), Pt(praw[t][:level + 1], level, 2.0 ** 25))
            acc = term if acc is None else orc.add(acc, term)
        assert outs[o].scale == 2.0 ** 55
        assert np.array_equal(ctx.ct_to_coeff(outs[o]), acc.data), o


def test_batched_errors_and_empty():
    from paper_2509_22857_amd import ckks
    from paper_2509_22857_amd.ckks import CkcError
    ps = tiny()
    ctx, orc, torch = _setup(ps)
    keys = ctx.keygen(3, [1])
    _, cts = _cts(ctx, ps, (1, 2), 2)
    assert ckks.rotate_many(ctx, keys, [], [1], outs=[]) == []
    with pytest.raises(CkcError) as e:
        ckks.rotate_many(ctx, keys, cts, [5])
    assert e.value.code == -4
    low = ctx.mod_drop(cts[1], 1)
    with pytest.raises(CkcError) as e:
        ckks.mul_relin_many(ctx, keys, [cts[0], low], [cts[0], low])
    assert e.value.code == -2
    pts = [ctx.pt_from_coeff(gen.random_limbs(5, ps.q, ps.N), 2, 1.0)] * 65
    with pytest.raises(CkcError) as e:
        ckks.mac_plain_many(ctx, cts * 33, pts[:65])
    assert e.value.code == -1
    lowpt = ctx.pt_from_coeff(gen.random_limbs(6, ps.q, ps.N), 1, 1.0)
    with pytest.raises(CkcError) as e:
        ckks.mac_plain_many(ctx, cts[:1], [lowpt])
    assert e.value.code == -2


def test_stream_reserve_and_release_keep_results():
    """A stream whose arena was reserved up front, or freed between calls,
    gives the same bits as the default stream; a reservation the device
    cannot hold is refused with CKC_ENOMEM and leaves the stream usable."""
    from paper_2509_22857_amd import ckks
    ps = tiny()
    ctx, orc, torch = _setup(ps)
    keys = ctx.keygen(5, [1, -3])
    _, cts = _cts(ctx, ps, range(300, 306), 2)
    ref = [o.buf.clone() for o in ckks.rotate_many(ctx, keys, cts, [1, -3])]
    s = torch.cuda.Stream()
    ckks.stream_reserve(1 << 26, s)
    for rnd in range(2):
        with torch.cuda.stream(s):
            got = ckks.rotate_many(ctx, keys, cts, [1, -3], stream=s)
        s.synchronize()
        assert all(torch.equal(g.buf, r) for g, r in zip(got, ref)), rnd
        ckks.stream_release(s)
    with pytest.raises(ckks.CkcError, match="CKC_ENOMEM"):
        ckks.stream_reserve(1 << 52, s)
    with torch.cuda.stream(s):
        got = ckks.rotate_many(ctx, keys, cts, [1, -3], stream=s)
    s.synchronize()
    assert all(torch.equal(g.buf, r) for g, r in zip(got, ref))
    ckks.stream_release(s)
