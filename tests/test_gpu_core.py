"""GPU <-> oracle parity of the RNS-CKKS primitives, through the C-ABI.

Every comparison is bit-exact in coefficient form (the GPU keeps ciphertexts
in NTT form; the test converts them back with the library's own inverse NTT,
whose correctness is pinned separately against direct evaluation).
"""
import numpy as np
import pytest

from workloads import gen
from workloads.params import tiny, mid, micro

pytestmark = pytest.mark.gpu


def _bitrev(x, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r


def _eval(a, x, q):
    v = 0
    for c in reversed([int(t) for t in a]):
        v = (v * x + c) % q
    return v


@pytest.fixture(scope="module", params=["tiny", "mid", "micro"])
def env(request):
    import torch
    from paper_2509_22857_amd.ckks import Context
    from oracle.ckks import Oracle
    ps = {"tiny": tiny, "mid": mid, "micro": micro}[request.param]()
    print(f"[env] params={ps.name} N={ps.N} nq={len(ps.q)} np={len(ps.p)}", flush=True)
    ctx = Context.from_params(ps)
    orc = Oracle.from_params(ps)
    return ps, ctx, orc, torch


def test_ntt_evaluation_order_and_roundtrip(env):
    ps, ctx, orc, torch = env
    nl = len(ps.q)
    a = gen.random_limbs(101, ps.q, ps.N)
    buf = ctx.upload_words(a)
    ctx.ntt(buf, 1, nl, False)
    torch.cuda.synchronize()
    A = ctx.download_words(buf).reshape(nl, ps.N)
    for l in (0, nl - 1):
        q, psi = ps.q[l], ctx.root(l)
        assert pow(psi, ps.N, q) == q - 1
        for k in (0, 1, ps.N // 2 + 3, ps.N - 1):
            assert int(A[l, k]) == _eval(a[l], pow(psi, 2 * _bitrev(k, ps.logN) + 1, q), q)
    ctx.ntt(buf, 1, nl, True)
    torch.cuda.synchronize()
    assert np.array_equal(ctx.download_words(buf).reshape(nl, ps.N), a)


def test_mul_plain_matches_oracle_products(env):
    ps, ctx, orc, torch = env
    level = len(ps.q) - 1 if ps.name == "tiny" else min(3, len(ps.q) - 1)
    ct = gen.random_ct(7, ps.q, level, ps.N)
    pt = gen.random_limbs(8, ps.q[:level + 1], ps.N)
    g = ctx.mul_plain(ctx.ct_from_coeff(ct, level, 1.0), ctx.pt_from_coeff(pt, level, 1.0))
    got = ctx.ct_to_coeff(g)
    from oracle.ckks import Ct, Pt
    want = orc.mul_plain(Ct(ct, level, 1.0), Pt(pt, level, 1.0))
    assert np.array_equal(got, want.data)


def test_secret_encode_encrypt_bit_exact(env):
    ps, ctx, orc, torch = env
    seed = 4242
    keys = ctx.keygen(seed, [])
    sk = orc.secret_key(seed)
    level = len(ps.q) - 1
    z = gen.uniform_slots(5, ps.N // 2)
    pt = ctx.encode(z, level, 2.0 ** 40)
    opt = orc.encode(z, level, 2.0 ** 40)
    assert np.array_equal(ctx.pt_to_coeff(pt), opt.data)
    ct = ctx.encrypt(keys, pt, 77)
    oct_ = orc.encrypt(opt, sk, 77)
    assert np.array_equal(ctx.ct_to_coeff(ct), oct_.data)
    dec = ctx.decrypt(keys, ct)
    assert np.array_equal(ctx.pt_to_coeff(dec), orc.decrypt(oct_, sk))
    zz = ctx.decode(dec)
    assert np.max(np.abs(zz - z)) < 1e-6
    assert np.max(np.abs(zz - orc.decode(orc.decrypt(oct_, sk), oct_.scale))) < 1e-9


def test_encode_encrypt_image_matches_oracle(env):
    """One-call HW packing + encryption of an image: channel c equals the
    oracle's encryption (stream stream_id + c) of the slot vector with every
    member block holding the image at row stride W0."""
    ps, ctx, orc, torch = env
    if ps.N < 2 ** 12 or ps.name == "micro":
        pytest.skip("one small and one mid parameter set suffice")
    seed = 99
    keys = ctx.keygen(seed, [])
    sk = orc.secret_key(seed)
    level = len(ps.q) - 1
    Cn, H, W, M, B, W0 = 3, 6, 5, 2, 64, 8
    img = gen.images(3, 1, Cn, H, W)[0]
    cts = ctx.encode_encrypt_image(keys, img, M, B, W0, level, 2.0 ** 30, 5000)
    assert len(cts) == Cn
    for c in range(Cn):
        z = np.zeros(M * B)
        for m in range(M):
            for r in range(H):
                z[m * B + r * W0: m * B + r * W0 + W] = img[c, r]
        want = orc.encrypt(orc.encode(z, level, 2.0 ** 30), sk, 5000 + c)
        assert cts[c].level == level and cts[c].scale == 2.0 ** 30
        assert np.array_equal(ctx.ct_to_coeff(cts[c]), want.data), c
    from paper_2509_22857_amd.ckks import CkcError
    with pytest.raises(CkcError, match="CKC_EINVAL"):
        ctx.encode_encrypt_image(keys, img, M, 16, W0, level, 2.0 ** 30, 5000)  # rows overflow the block


def test_encode_bit_exact_at_large_scales(env):
    """Encodings at scales where the FFT's last bits decide the integers."""
    ps, ctx, orc, torch = env
    level = min(2, len(ps.q) - 1)
    n = ps.N // 2
    z = gen.uniform_slots(31, n, -3, 3)
    blk = np.zeros(n)
    blk[: n // 4] = 0.37
    blk[n // 4: n // 2] = -1.25
    for vec in (z, blk):
        for scale in (2.0 ** 30, 2.0 ** 60, 2.0 ** 90):
            got = ctx.pt_to_coeff(ctx.encode(vec, level, scale))
            assert np.array_equal(got, orc.encode(vec, level, scale).data), scale


def test_tensor_relin_rescale_bit_exact(env):
    ps, ctx, orc, torch = env
    from oracle.ckks import Ct
    seed = 99
    keys = ctx.keygen(seed, [])
    sk = orc.secret_key(seed)
    level = len(ps.q) - 1 if ps.name == "tiny" else min(5, len(ps.q) - 1)
    a = gen.random_ct(11, ps.q, level, ps.N)
    b = gen.random_ct(12, ps.q, level, ps.N)
    ga, gb = ctx.ct_from_coeff(a, level, 2.0 ** 40), ctx.ct_from_coeff(b, level, 2.0 ** 40)
    t = ctx.tensor(ga, gb)
    ot = orc.tensor(Ct(a, level, 2.0 ** 40), Ct(b, level, 2.0 ** 40))
    assert np.array_equal(ctx.ct_to_coeff(t), ot.data)
    r = ctx.relin(keys, t)
    orr = orc.relin(ot, orc.relin_key(sk))
    assert np.array_equal(ctx.ct_to_coeff(r), orr.data)
    rs = ctx.rescale(r)
    ors = orc.rescale(orr)
    assert rs.level == ors.level and rs.scale == ors.scale
    assert np.array_equal(ctx.ct_to_coeff(rs), ors.data)


def test_hoisted_rotations_bit_exact(env):
    ps, ctx, orc, torch = env
    from oracle.ckks import Ct
    seed = 5
    steps = [1, -1, 31, 0] if ps.name == "tiny" else [1, -33]
    keys = ctx.keygen(seed, steps)
    sk = orc.secret_key(seed)
    level = len(ps.q) - 1 if ps.name == "tiny" else min(4, len(ps.q) - 1)
    a = gen.random_ct(13, ps.q, level, ps.N)
    outs = ctx.rotate(keys, ctx.ct_from_coeff(a, level, 1.0), steps)
    for r, o in zip(steps, outs):
        g = orc.galois_elt(r)
        gk = orc.galois_key(sk, g) if g != 1 else None
        want = orc.rotate(Ct(a, level, 1.0), r, gk)
        assert np.array_equal(ctx.ct_to_coeff(o), want.data), r


def test_add_const_mod_drop_add_plain(env):
    ps, ctx, orc, torch = env
    from oracle.ckks import Ct, Pt
    level = len(ps.q) - 1 if ps.name == "tiny" else min(3, len(ps.q) - 1)
    a = gen.random_ct(21, ps.q, level, ps.N)
    b = gen.random_ct(22, ps.q, level, ps.N)
    s = 2.0 ** 70
    ga = ctx.ct_from_coeff(a, level, s)
    gc = ctx.add_const(ga, -0.3125)
    assert np.array_equal(ctx.ct_to_coeff(gc), orc.add_const(Ct(a, level, s), -0.3125).data)
    gs = ctx.sub(ga, ctx.ct_from_coeff(b, level, s))
    assert np.array_equal(ctx.ct_to_coeff(gs), orc.sub(Ct(a, level, s), Ct(b, level, s)).data)
    p = gen.random_limbs(23, ps.q[:level + 1], ps.N)
    gp = ctx.add_plain(ga, ctx.pt_from_coeff(p, level, s))
    assert np.array_equal(ctx.ct_to_coeff(gp), orc.add_plain(Ct(a, level, s), Pt(p, level, s)).data)
    gd = ctx.mod_drop(ga, level - 1)
    assert np.array_equal(ctx.ct_to_coeff(gd), orc.mod_drop(Ct(a, level, s), level - 1).data)


def test_errors_are_reported(env):
    ps, ctx, orc, torch = env
    from paper_2509_22857_amd.ckks import CkcError
    level = 1
    a = ctx.ct_from_coeff(gen.random_ct(1, ps.q, level, ps.N), level, 1.0)
    b = ctx.ct_from_coeff(gen.random_ct(2, ps.q, level, ps.N), level, 2.0)
    with pytest.raises(CkcError) as e:
        ctx.add(a, b)
    assert e.value.code == -3
    keys = ctx.keygen(1, [])
    with pytest.raises(CkcError) as e:
        ctx.rotate(keys, a, [3])
    assert e.value.code == -4
    z = ctx.mod_drop(a, 0)
    with pytest.raises(CkcError) as e:
        ctx.rescale(z)
    assert e.value.code == -2


def test_library_loaded_and_context_created_before_torch_uses_the_device():
    """Loading the library and creating a context before anything of torch
    has touched the GPU leaves torch usable (the binding loads torch's HIP
    runtime before the library's), and creating the context loads no code
    object."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2509_22857_amd import ckks\n"
            "ckks.lib()\n"
            "from workloads.params import tiny\n"
            "ctx = ckks.Context.from_params(tiny())\n"
            "import torch\n"
            "x = torch.ones(4, device='cuda'); torch.cuda.current_stream().synchronize()\n"
            "keys = ctx.keygen(3, [1])\n"
            "torch.cuda.synchronize(); print('ok', float(x.sum()))\n") % root
    print("[ordering] library and context before torch's device set-up, in a child process", flush=True)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "ok 4.0" in r.stdout, r.stdout + r.stderr
