"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against mathematics that fixes the answer: the
O(N^2) schoolbook negacyclic product, direct evaluation at roots of unity,
the O(N^2) definition of the canonical embedding, big-integer CRT identities
for ModUp / ModDown / rescale, composition of automorphisms, the published
SplitMix64 test vector, and decryption-level identities.
"""
import json
import os

import numpy as np
import pytest

from oracle.ckks import Oracle, Pt, Ct, lib
from workloads.params import balanced_chain, nearest_prime, is_prime, tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_oracle(logN=6, bits=(40, 40, 40), pbits=(50,), alpha=1):
    two_n = 2 << logN
    q = balanced_chain(list(bits), two_n)
    p = balanced_chain(list(pbits), two_n, exclude=q)
    return Oracle(logN, q, p, alpha)


def schoolbook_negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            v = ai * int(b[j])
            if k < n:
                out[k] += v
            else:
                out[k - n] -= v
    return np.array([x % q for x in out], dtype=np.uint64)


def crt(residues, mods):
    """Integer in [0, prod) with the given residues (Python big ints)."""
    M = 1
    for m in mods:
        M *= m
    x = 0
    for r, m in zip(residues, mods):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M, M


def centred(x, M):
    return x - M if x > M // 2 else x


# --------------------------------------------------------------- PRNG


def test_splitmix64_published_vector():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    got = [lib().oc_draw(g["state"], j) for j in range(len(g["outputs"]))]
    assert got == [int(x) for x in g["outputs"]]


def test_samplers_moments():
    o = small_oracle(logN=12)
    sk = o.secret_key(7)
    s = sk.s.astype(np.int64)
    assert set(np.unique(s)) <= {-1, 0, 1}
    freq = np.array([(s == v).mean() for v in (-1, 0, 1)])
    assert np.all(np.abs(freq - 1 / 3) < 0.03)
    # encryption error: decrypt(encrypt(0)) is the centred-binomial error
    pt = Pt(np.zeros((3, o.N), dtype=np.uint64), 2, 1.0)
    ct = o.encrypt(pt, sk, 11)
    m = o.decrypt(ct, sk)
    e = np.array([centred(int(x), o.q[0]) for x in m[0]])
    assert np.all(np.abs(e) <= 21)
    assert abs(e.mean()) < 0.3 and abs(e.var() - 10.5) < 1.5
    # same error on every limb (one draw per coefficient)
    for l in range(1, 3):
        el = np.array([centred(int(x), o.q[l]) for x in m[l]])
        assert np.array_equal(el, e)


# --------------------------------------------------------------- primes


def test_paper_chains_reproduced():
    g = json.load(open(os.path.join(GOLDEN, "paper_moduli.json")))
    for name, c in g["chains"].items():
        qs = [int(x, 16) for x in c["q"]]
        two_n = 2 << c["logN"]
        main = balanced_chain(c["sizes"], two_n)
        assert main == qs[:-1], name
        for q in qs + [int(c["P"], 16)]:
            assert is_prime(q) and (q - 1) % two_n == 0, (name, hex(q))
        log2q = sum(np.log2(float(q)) for q in qs)
        assert abs(log2q - c["log2Q"]) < 1.0, name


def test_prime_sets_valid():
    for ps in (tiny(),):
        two_n = 2 * ps.N
        allp = list(ps.q) + list(ps.p)
        assert len(set(allp)) == len(allp)
        for q in allp:
            assert is_prime(q) and (q - 1) % two_n == 0 and q < (1 << 62)


# --------------------------------------------------------------- NTT


@pytest.mark.parametrize("logN", [3, 5, 7])
def test_ntt_product_vs_schoolbook(logN):
    o = small_oracle(logN=logN, bits=(40, 50, 60), pbits=(61,))
    rng = np.random.default_rng(logN)
    for t, q in enumerate(o.mod):
        a = rng.integers(0, q, o.N, dtype=np.uint64)
        b = rng.integers(0, q, o.N, dtype=np.uint64)
        assert np.array_equal(o.polymul(a, b, t), schoolbook_negacyclic(a, b, q))


def test_ntt_is_evaluation_at_odd_powers():
    o = small_oracle(logN=6, bits=(50,), pbits=(55,))
    rng = np.random.default_rng(1)
    for t, q in enumerate(o.mod):
        a = rng.integers(0, q, o.N, dtype=np.uint64)
        A = o.ntt(a, t)
        psi = o.psi(t)
        assert pow(psi, o.N, q) == q - 1
        for k in (0, 1, 5, o.N - 1):
            x = pow(psi, 2 * k + 1, q)
            val = 0
            for c in reversed([int(v) for v in a]):
                val = (val * x + c) % q
            assert int(A[k]) == val
        assert np.array_equal(o.intt(A, t), a)


# --------------------------------------------------------------- automorphism


def test_automorphism_composition():
    o = small_oracle(logN=8)
    rng = np.random.default_rng(2)
    a = rng.integers(0, o.q[0], o.N, dtype=np.uint64)
    two_n = 2 * o.N
    for g, h in ((5, 25), (3, 7), (5, two_n - 1), (o.galois_elt(-1), 5)):
        lhs = o.automorphism(o.automorphism(a, h, 0), g, 0)
        rhs = o.automorphism(a, (g * h) % two_n, 0)
        assert np.array_equal(lhs, rhs)
    # sigma_g is a ring homomorphism: sigma(a b) = sigma(a) sigma(b)
    b = rng.integers(0, o.q[0], o.N, dtype=np.uint64)
    g = 5
    assert np.array_equal(o.automorphism(o.polymul(a, b, 0), g, 0),
                          o.polymul(o.automorphism(a, g, 0), o.automorphism(b, g, 0), 0))


def test_galois_element_of_inverse_rotation():
    o = small_oracle(logN=8)
    two_n = 2 * o.N
    for r in (1, 3, 17):
        assert (o.galois_elt(r) * o.galois_elt(-r)) % two_n == 1


# --------------------------------------------------------------- encoding


@pytest.mark.parametrize("logN", [4, 6, 9])
def test_encoding_matches_embedding_definition(logN):
    o = small_oracle(logN=logN)
    N, n = o.N, o.N // 2
    rng = np.random.default_rng(logN)
    z = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    w = o.encode_w(z)
    # definition: m_k = (2/N) Re sum_j z_j zeta^(-k 5^j), zeta = exp(i pi / N)
    e = np.array([pow(5, j, 2 * N) for j in range(n)])
    k = np.arange(N)
    zeta = np.exp(-1j * np.pi * np.outer(k, e) / N)
    m_def = (2.0 / N) * np.real(zeta @ z)
    assert np.max(np.abs(w - m_def)) < 1e-12
    # and the slots are the polynomial evaluated at zeta^(5^j)
    roots = np.exp(1j * np.pi * e / N)
    evals = np.array([np.polyval(w[::-1], r) for r in roots])
    assert np.max(np.abs(evals - z)) < 1e-10


def test_encode_decode_roundtrip_and_constant():
    o = small_oracle(logN=10, bits=(60, 40, 40))
    n = o.N // 2
    rng = np.random.default_rng(3)
    z = rng.uniform(-3, 3, n)
    pt = o.encode(z, 2, 2.0 ** 30)
    assert np.max(np.abs(o.decode(pt.data, pt.scale) - z)) < 1e-6
    # the constant vector encodes to the constant polynomial
    c = o.encode(np.full(n, 0.75), 0, 2.0 ** 20)
    assert int(c.data[0, 0]) == round(0.75 * 2 ** 20)
    assert np.all(c.data[0, 1:] == 0)


def test_canonical_twiddles_match_libm():
    """The series-based twiddles used by the encoding FFT equal cos/sin to
    within a few ulp over every table the transforms use."""
    import ctypes as C
    L = lib()
    L.oc_canon_cs.argtypes = [C.c_uint64, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    c, s = C.c_double(), C.c_double()
    for M in (1 << 12, 1 << 16, 1 << 17):
        js = list(range(0, M // 2, max(1, M // 4096))) + [M // 8, M // 4, 3 * M // 8, M // 2 - 1]
        for j in js:
            L.oc_canon_cs(j, M, C.byref(c), C.byref(s))
            ang = 2 * np.pi * j / M
            assert abs(c.value - np.cos(ang)) < 1e-15 and abs(s.value - np.sin(ang)) < 1e-15, (j, M)


def test_const_residue_of_large_values():
    o = small_oracle(logN=4, bits=(60, 61, 40))
    v, s = -0.3125, 2.0 ** 90
    r = o.const_residues(v, s, 3)
    exact = round(v * s)  # v*s is exact in double; Python int
    for t in range(3):
        assert int(r[t]) == exact % o.q[t]


# --------------------------------------------------------------- RNS identities


def test_modup_identity_bigint():
    """ModUp of digit j lifts the digit to its centred representative plus
    u Q_j with |u| < |D_j|/2: X (the value over the extended basis, centred)
    is congruent to the digit mod Q_j, |X| < |D_j| Q_j / 2, and X / Q_j has
    mean ~0 (a lift over [0, Q_j) has mean about |D_j|/2 and fails here)."""
    o = small_oracle(logN=7, bits=(40, 41, 42, 43, 44), pbits=(61, 61), alpha=2)
    rng = np.random.default_rng(4)
    level = 4
    d = np.stack([rng.integers(0, q, o.N, dtype=np.uint64) for q in o.q])
    ext_mods = o.q[:level + 1] + o.p
    M = 1
    for m in ext_mods:
        M *= m
    for j in range(3):
        lo, hi = 2 * j, min(2 * j + 1, level)
        D = o.q[lo:hi + 1]
        Qj = 1
        for x in D:
            Qj *= x
        up = o.modup_digit(d, level, j)
        ratios = []
        for k in range(o.N):
            X, _ = crt([up[t, k] for t in range(len(ext_mods))], ext_mods)
            if X > M // 2:
                X -= M
            dhat, _ = crt([d[i, k] for i in range(lo, hi + 1)], D)
            assert X % Qj == dhat
            assert 2 * abs(X) < len(D) * Qj
            ratios.append(X / Qj)
        assert abs(np.mean(ratios)) < 0.1 * len(D)


@pytest.mark.parametrize("bits,pbits", [((40, 41, 42), (60, 61)), ((50, 51, 52), (40, 41, 42))])
def test_moddown_is_unbiased_rounded_division_bigint(bits, pbits):
    """ModDown divides by P with rounding to the nearest integer up to the
    fast conversion's carry, which is centred: with X the value of x over
    Q u P, E = x - y P over Q is a lift of x_P with |E| < n_P P / 2, so
    |y - X/P| < (n_P + 1)/2, and the error y - X/P has mean ~0 (a floor-type
    conversion over [0, p_k) has mean about -(n_P/2) and fails here)."""
    o = small_oracle(logN=8, bits=bits, pbits=pbits, alpha=1)
    rng = np.random.default_rng(5)
    level = 2
    ext = o.q[:level + 1] + o.p
    x = np.stack([rng.integers(0, m, o.N, dtype=np.uint64) for m in ext])
    y = o.moddown(x, level)
    P = 1
    for pa in o.p:
        P *= pa
    Q = o.q[0] * o.q[1] * o.q[2]
    errs = []
    for k in range(o.N):
        E, _ = crt([(int(x[i, k]) - int(y[i, k]) * P) % o.q[i] for i in range(level + 1)], o.q[:level + 1])
        if E > Q // 2:
            E -= Q
        for a, pa in enumerate(o.p):
            assert E % pa == int(x[level + 1 + a, k])
        assert 2 * abs(E) < len(o.p) * P
        X, _ = crt([int(x[t, k]) for t in range(len(ext))], ext)
        Y, _ = crt([int(y[i, k]) for i in range(level + 1)], o.q[:level + 1])
        d = (Y - X // P) % Q  # y - floor(X / P), as a small centred integer
        if d > Q // 2:
            d -= Q
        errs.append(d - (X % P) / P)
    errs = np.array(errs)
    assert np.max(np.abs(errs)) < (len(o.p) + 1) / 2
    assert abs(errs.mean()) < 0.1


def test_rescale_is_rounded_division_bigint():
    o = small_oracle(logN=5, bits=(50, 45, 40))
    rng = np.random.default_rng(6)
    ct = Ct(np.stack([np.stack([rng.integers(0, q, o.N, dtype=np.uint64) for q in o.q])
                      for _ in range(2)]), 2, 2.0 ** 40)
    out = o.rescale(ct)
    Q = o.q[0] * o.q[1] * o.q[2]
    Qp = o.q[0] * o.q[1]
    ql = o.q[2]
    for p in range(2):
        for k in range(o.N):
            X, _ = crt([ct.data[p, l, k] for l in range(3)], o.q)
            Xc = centred(X, Q)
            want = (2 * Xc + ql) // (2 * ql)  # round half up; q odd so no ties
            Y, _ = crt([out.data[p, l, k] for l in range(2)], o.q[:2])
            assert centred(Y, Qp) == want


# --------------------------------------------------------------- decryption-level


def _setup_tiny():
    ps = tiny()
    o = Oracle.from_params(ps)
    sk = o.secret_key(1234)
    return o, sk


def test_encrypt_decrypt_exact():
    o, sk = _setup_tiny()
    rng = np.random.default_rng(8)
    z = rng.uniform(-1, 1, o.N // 2)
    pt = o.encode(z, o.L, 2.0 ** 40)
    ct = o.encrypt(pt, sk, 3)
    m = o.decrypt(ct, sk)
    for l in range(o.L + 1):
        diff = (m[l].astype(object) - pt.data[l].astype(object)) % o.q[l]
        e = np.array([centred(int(v), o.q[l]) for v in diff])
        assert np.all(np.abs(e) <= 21)
    assert np.max(np.abs(o.decode(m, ct.scale) - z)) < 1e-6


@pytest.mark.slow
def test_relin_and_rotation_decrypt_tiny():
    o, sk = _setup_tiny()
    rng = np.random.default_rng(9)
    n = o.N // 2
    z1, z2 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    c1 = o.encrypt(o.encode(z1, o.L, 2.0 ** 40), sk, 1)
    c2 = o.encrypt(o.encode(z2, o.L, 2.0 ** 40), sk, 2)
    rlk = o.relin_key(sk)
    prod = o.relin(o.tensor(c1, c2), rlk)
    res = o.decrypt_decode(o.rescale(prod), sk)
    assert np.max(np.abs(res - z1 * z2)) < 1e-4
    for r in (1, -3, 64):
        gk = o.galois_key(sk, o.galois_elt(r))
        rot = o.decrypt_decode(o.rotate(c1, r, gk), sk)
        assert np.max(np.abs(rot - np.roll(z1, -r))) < 1e-4
    # rotation composition (semantic)
    g1, g2 = o.galois_elt(1), o.galois_elt(2)
    k1, k2 = o.galois_key(sk, g1), o.galois_key(sk, g2)
    both = o.rotate(o.rotate(c1, 1, k1), 1, k1)
    assert np.max(np.abs(o.decrypt_decode(both, sk) - o.decrypt_decode(o.rotate(c1, 2, k2), sk))) < 1e-4


def test_keyswitch_noise_bound_tiny():
    """u0 + u1 s - d s' is small (key-switching noise), checked exactly."""
    o, sk = _setup_tiny()
    rng = np.random.default_rng(10)
    level = o.L
    d = np.stack([rng.integers(0, q, o.N, dtype=np.uint64) for q in o.q])
    rlk = o.relin_key(sk)
    u = o.keyswitch(d, level, rlk, 1)
    sl = o.secret_limbs(sk)
    for l in range(level + 1):
        q = o.q[l]
        s2 = o.polymul(sl[l], sl[l], l)
        lhs = (u[0, l].astype(object) + o.polymul(u[1, l], sl[l], l).astype(object)) % q
        rhs = o.polymul(d[l], s2, l).astype(object)
        err = np.array([centred(int(v), q) for v in (lhs - rhs) % q])
        assert np.max(np.abs(err)) < 2 ** 20


def test_mul_const_equals_product_with_encoded_constant_vector():
    """Section 2.2: the encoding of the all-w slot vector is the constant
    polynomial round(w * scale); multiplying by it limb-wise (mul_const) must
    equal the negacyclic product with that encoded plaintext."""
    from oracle.ckks import Oracle, Ct
    from workloads import gen
    from workloads.params import tiny
    ps = tiny()
    o = Oracle.from_params(ps)
    level = len(ps.q) - 1
    a = Ct(gen.random_ct(41, ps.q, level, ps.N), level, 2.0 ** 20)
    for w, sc in ((0.37, 2.0 ** 30), (-1.25, 2.0 ** 40), (3.0e-3, 2.0 ** 55)):
        p = o.encode(np.full(ps.N // 2, w), level, sc)
        assert not p.data[:, 1:].any()
        want = o.mul_plain(a, p)
        got = o.mul_const(a, w, sc)
        assert got.scale == want.scale
        assert np.array_equal(got.data, want.data)


def test_keyswitch_ext_then_moddown_is_the_keyswitch():
    """Section 2.2 hybrid key switching: the extended-basis product followed
    by ModDown is the key switch; ModDown of (P x, 0) is x exactly."""
    from oracle.ckks import Oracle
    from workloads import gen
    from workloads.params import small_tower
    ps = small_tower(logN=12, levels=3)
    o = Oracle.from_params(ps)
    sk = o.secret_key(3)
    level = 2
    d = gen.random_limbs(5, ps.q[:level + 1], ps.N)
    g = o.galois_elt(5)
    key = o.galois_key(sk, g)
    ext = o.keyswitch_ext(d, level, key, g)
    want = o.keyswitch(d, level, key, g)
    for b in range(2):
        assert np.array_equal(o.moddown(ext[b], level), want[b])
    nl = level + 1
    x = gen.random_limbs(6, ps.q[:nl], ps.N)
    px = np.zeros((nl + len(ps.p), ps.N), dtype=np.uint64)
    for l in range(nl):
        P = 1
        for pk in ps.p:
            P = P * pk % ps.q[l]
        px[l] = ((x[l].astype(object) * P) % ps.q[l]).astype(np.uint64)
    assert np.array_equal(o.moddown(px, level), x)


def test_double_hoisted_convolution_decrypts_to_the_convolution():
    """The convolution summed in the extended basis with one ModDown per
    output decrypts to the exact (FP64) convolution of the image within the
    input's encryption noise; rotations that each run their own ModDown
    before the plaintext products (a different ciphertext) carry the ModDown
    rounding of every rotation into the result and land further away."""
    from oracle.ckks import Oracle
    from oracle.network import OracleNetwork
    from workloads import gen
    from workloads.params import small_tower
    ps = small_tower(logN=12, levels=3, alpha=1)  # one prime per digit: negligible key-switching noise
    o = Oracle.from_params(ps)
    g = np.random.default_rng(2)
    I, O, k = 2, 2, 4
    cb = g.uniform(-0.5, 0.5, (3, k, 1))
    idx = g.integers(0, k, (O, I, 3, 3)).astype(np.uint16)
    spec = dict(name="c", members=1, classes=0, image=(I, 8, 8), layout=dict(block=64, row_stride=8),
                layers=[dict(op="conv", name="conv", inp="x", out="c", out_ch=O, in_ch=I, ksize=3, stride=1,
                             codebook=cb, idx=idx, bias=None)], k=k)
    D = 2.0 ** 30
    net = OracleNetwork(o, spec, D, D, D)
    sk = o.secret_key(8)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps()}
    img = gen.images(3, 1, I, 8, 8)[0]
    xs = net.encrypt_image(sk, img, 10)
    level = xs[0].level
    outs, grid = net.conv(xs, dict(gap=1, H=8, W=8), spec["layers"][0], D, 1.0, gk, with_bias=False)
    for oc in range(O):
        exact = np.zeros((8, 8))
        ref = None
        for i in range(I):
            for dh in (-1, 0, 1):
                for dw in (-1, 0, 1):
                    w = cb[dw + 1][idx[oc, i, dh + 1, dw + 1]][0]
                    st = dh * 8 + dw
                    v = np.zeros(ps.N // 2)
                    for rr in range(8):
                        for cc in range(8):
                            if 0 <= rr + dh < 8 and 0 <= cc + dw < 8:
                                exact[rr, cc] += w * img[i, rr + dh, cc + dw]
                                v[rr * 8 + cc] = w
                    r = o.rotate(xs[i], st, gk.get(o.galois_elt(st)))
                    t = o.mul_plain(r, o.encode(v, level, D))
                    ref = t if ref is None else o.add(ref, t)
        got = o.decrypt_decode(outs[oc], sk)[:64].reshape(8, 8)
        per_rot = o.decrypt_decode(ref, sk)[:64].reshape(8, 8)
        assert not np.array_equal(outs[oc].data, ref.data)
        assert np.max(np.abs(got - exact)) < 2e-6
        assert np.max(np.abs(per_rot - exact)) < 1e-4


def test_key_switch_error_is_not_heavy_tailed_in_the_slots():
    """A rotation's decryption error, slot by slot, is spread like noise
    (largest slot about 6x the mean at N = 2^12): the key switch's digits and
    its division by P are centred.  With digits lifted over [0, Q_j) the error
    gathers a constant-times-sum term whose canonical embedding peaks in the
    slots near 1 (ratio near 50 here, growing like N^1.5)."""
    from workloads import gen
    from workloads.params import resnet20_tower, ParamSet
    base = resnet20_tower()
    ps = ParamSet("t", 12, base.q, base.p, alpha=3, delta_log2=30)
    o = Oracle.from_params(ps)
    sk = o.secret_key(9)
    z = gen.uniform_slots(5, ps.N // 2)
    ct = o.encrypt(o.encode(z, o.L, 2.0 ** 30), sk, 3)
    g = o.galois_elt(1)
    r = o.rotate(ct, 1, o.galois_key(sk, g))
    e = np.abs(o.decrypt_decode(r, sk) - np.roll(z, -1))
    assert e.max() < 12 * e.mean()
