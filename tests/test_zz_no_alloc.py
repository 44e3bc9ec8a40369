"""The relinearisation that allocates nothing (its scratch in the library's
static device array) gives ckc_relin's result bit for bit, on two calls in a
row with the second on a smaller ciphertext, and refuses a ciphertext that
needs more scratch than the array holds."""
import numpy as np
import pytest

from workloads import gen
from workloads.params import micro, balanced_chain, ParamSet

pytestmark = pytest.mark.gpu


def test_relin_noalloc_matches_relin_twice_then_smaller():
    from paper_2509_22857_amd import ckks
    from paper_2509_22857_amd.ckks import Context
    ps = micro()
    print("[no_alloc] micro N=2^16, 24+3 primes, levels 23 then 9", flush=True)
    ctx = Context.from_params(ps)
    keys = ctx.keygen(91, [])
    cap = int(ckks.lib().ckc_noalloc_capacity())
    for call, level in enumerate((ps.L, 9)):
        need = int(ckks.lib().ckc_relin_noalloc_bytes(ctx.h, level))
        assert 0 < need <= cap, (level, need, cap)
        z = gen.uniform_slots(300 + call, ps.N // 2)
        ct = ctx.encrypt(keys, ctx.encode(z, level, 2.0 ** 40), 50 + call)
        t = ctx.tensor(ct, ct)
        want = ctx.relin(keys, t)
        got = ctx.new_ct(level, 2)
        got.buf.fill_(-1)
        ctx.relin_noalloc(keys, t, got)
        assert got.level == want.level and got.npoly == 2 and got.scale == want.scale
        assert np.array_equal(got.buf.cpu().numpy(), want.buf.cpu().numpy()), (call, level)


def test_relin_noalloc_refuses_what_does_not_fit():
    from paper_2509_22857_amd import ckks
    from paper_2509_22857_amd.ckks import Context
    two_n = 2 << 16
    q = balanced_chain([60] * 40, two_n)
    p = balanced_chain([61] * 3, two_n, exclude=q)
    ps = ParamSet("wide", 16, tuple(q), tuple(p), alpha=3, delta_log2=40)
    print("[no_alloc] N=2^16, 40+3 primes: scratch beyond the static array", flush=True)
    ctx = Context.from_params(ps)
    need = int(ckks.lib().ckc_relin_noalloc_bytes(ctx.h, ps.L))
    assert need > int(ckks.lib().ckc_noalloc_capacity())
    keys = ctx.keygen(92, [])
    ct = ctx.encrypt(keys, ctx.encode(gen.uniform_slots(5, ps.N // 2), ps.L, 2.0 ** 40), 1)
    t = ctx.tensor(ct, ct)
    out = ctx.new_ct(ps.L, 2)
    with pytest.raises(ckks.CkcError, match="CKC_ENOMEM"):
        ctx.relin_noalloc(keys, t, out)
