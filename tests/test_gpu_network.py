"""GPU network evaluation vs the oracle: bit-exact ciphertexts at every
layer, decryptions vs the FP64 forward, and batch independence."""
import numpy as np
import pytest

from workloads import gen, nets
from workloads.params import tiny, small_tower

pytestmark = pytest.mark.gpu


def _coeff(ctx, ct):
    return ctx.ct_to_coeff(ct)


def _setup(ps, spec, delta, target, in_scale, seed):
    from paper_2509_22857_amd.ckks import Context
    from paper_2509_22857_amd.network import GpuNetwork
    from oracle.ckks import Oracle
    from oracle.network import OracleNetwork
    ctx = Context.from_params(ps)
    gnet = GpuNetwork(ctx, spec, delta, target, in_scale)
    keys = ctx.keygen(seed, gnet.steps)
    o = Oracle.from_params(ps)
    onet = OracleNetwork(o, spec, delta, target, in_scale)
    assert sorted(onet.steps()) == gnet.steps
    sk = o.secret_key(seed)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in onet.steps()}
    return ctx, gnet, keys, o, onet, sk, rlk, gk


def test_tiny_network_bit_exact():
    ps = tiny()
    spec = nets.tiny_spec(0)
    print("[tiny_network] N=2^12 conv3x3+act", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, 2.0 ** 40, 2.0 ** 34, 2.0 ** 40, 77)
    img = gen.images(5, 1, 1, 8, 8)
    gin = gnet.encrypt_images(keys, img, 500)
    oin = onet.encrypt_image(sk, img[0], 500)
    for g, c in zip(gin[0], oin):
        assert np.array_equal(_coeff(ctx, g), c.data)
    gl, ol = [], []
    gout, _ = gnet.run(keys, gin, hook=lambda ly, outs: gl.append(_coeff(ctx, outs[0])))
    oout, grid = onet.run(sk, oin, rlk, gk, hook=lambda ly, outs: ol.append(outs[0].data))
    for a, b in zip(gl, ol):
        assert np.array_equal(a, b)
    from oracle.forward import forward
    ref = forward(spec, img[0])[0, 0]
    lay = gnet.layouts["y"]
    got = gnet.decrypt_grid(keys, gout[0][0], lay)[0]
    assert np.max(np.abs(got - ref)) < 1e-5


def test_small_resnet_ensemble_bit_exact_and_batch_independent():
    spec = nets.resnet_spec(seed=1, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16), k=8, calib=4)
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print("[small_resnet] N=2^12 M=2 widths=(4,8)", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 9)
    imgs = gen.images(3, 2, 3, 16, 16)
    gin = gnet.encrypt_images(keys, imgs, 100)
    # layer-by-layer capture for image 0 (first channel) in a batch of two
    gl = []
    gout, _ = gnet.run(keys, gin, hook=lambda ly, outs: gl.append((ly["name"], _coeff(ctx, outs[0]))))
    oin = onet.encrypt_image(sk, imgs[0], 100)
    ol = []
    oout, _ = onet.run(sk, oin, rlk, gk, hook=lambda ly, outs: ol.append((ly["name"], outs[0].data)))
    for (n1, a), (n2, b) in zip(gl, ol):
        assert n1 == n2
        assert np.array_equal(a, b), n1
    for k, (g, c) in enumerate(zip(gout[0], oout)):
        assert np.array_equal(_coeff(ctx, g), c.data), k
    # image 1 alone gives the same ciphertexts as in the batch
    alone, _ = gnet.run(keys, [gin[1]])
    for a, b in zip(alone[0], gout[1]):
        assert np.array_equal(_coeff(ctx, a), _coeff(ctx, b))
    from oracle.forward import forward
    for n in range(2):
        ref = forward(spec, imgs[n])
        got = gnet.decrypt_logits(keys, gout[n])
        assert np.max(np.abs(got - ref)) < 1e-3
        assert got.mean(0).argmax() == ref.mean(0).argmax()


def test_single_member_network_bit_exact():
    """One member: the dense layer multiplies by constants (the encoding of the
    constant slot vector) and the activation adds constants."""
    spec = nets.resnet_spec(seed=3, members=1, widths=(4,), blocks=1, classes=5, image=(3, 16, 16), k=4, calib=4)
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print("[single_member] N=2^12 M=1 widths=(4,)", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 21)
    imgs = gen.images(8, 1, 3, 16, 16)
    gin = gnet.encrypt_images(keys, imgs, 300)
    gl = []
    gout, _ = gnet.run(keys, gin, hook=lambda ly, outs: gl.append((ly["name"], _coeff(ctx, outs[0]))))
    oin = onet.encrypt_image(sk, imgs[0], 300)
    ol = []
    oout, _ = onet.run(sk, oin, rlk, gk, hook=lambda ly, outs: ol.append((ly["name"], outs[0].data)))
    for (n1, a), (n2, b) in zip(gl, ol):
        assert n1 == n2
        assert np.array_equal(a, b), n1
    for k, (g, c) in enumerate(zip(gout[0], oout)):
        assert np.array_equal(_coeff(ctx, g), c.data), k
    from oracle.forward import forward
    ref = forward(spec, imgs[0])
    got = gnet.decrypt_logits(keys, gout[0])
    assert np.max(np.abs(got - ref)) < 1e-3


def test_wide_conv_input_chunks_bit_exact():
    """A convolution with more input channels than one key-switching batch
    (70 = 64 + 6): the contraction accumulates per input chunk; stride 2 and
    a bias on top."""
    g = np.random.default_rng(4)
    I, O, k = 70, 9, 16
    codebook = g.uniform(-0.3, 0.3, (3, k, 1))
    idx = g.integers(0, k, (O, I, 3, 3)).astype(np.uint16)
    bias = g.uniform(-0.5, 0.5, (1, O))
    spec = dict(name="wide_conv", members=1, classes=0, image=(I, 8, 8), layout=dict(block=64, row_stride=8),
                layers=[dict(op="conv", name="conv", inp="x", out="c", out_ch=O, in_ch=I, ksize=3, stride=2,
                             codebook=codebook, idx=idx, bias=bias)], k=k)
    ps = small_tower(logN=12, levels=2)
    D = 2.0 ** 30
    print("[wide_conv] N=2^12 I=70 O=9 stride 2", flush=True)
    from paper_2509_22857_amd import ckks
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 5)
    imgs = gen.images(12, 2, I, 8, 8)
    gin = gnet.encrypt_images(keys, imgs, 700)
    want = []
    for n in range(2):
        oin = onet.encrypt_image(sk, imgs[n], 700 + n * 4096)
        oout, _ = onet.run(sk, oin, rlk, gk)
        assert len(oout) == O
        want.append([c.data for c in oout])
    # every launch form of the contraction: all output groups in one launch or
    # one launch per group, 8 or 16 outputs per wave
    saved = {k: ckks.tune_get(k) for k in ("conv_fuse", "conv_outs")}
    try:
        for fuse, outs in ((1, 8), (0, 8), (1, 16), (0, 16)):
            ckks.tune_set("conv_fuse", fuse)
            ckks.tune_set("conv_outs", outs)
            print(f"[wide_conv] conv_fuse={fuse} conv_outs={outs}", flush=True)
            gout, _ = gnet.run(keys, gin)
            for n in range(2):
                for j in range(O):
                    assert np.array_equal(_coeff(ctx, gout[n][j]), want[n][j]), (fuse, outs, n, j)
    finally:
        for k, v in saved.items():
            ckks.tune_set(k, v)


@pytest.mark.parametrize("hoist", [None, ["double", "single", "double", "single", "single"]])
def test_small_vgg_bit_exact(hoist):
    """VGG-style network (convolutions, activations, 2x2 sum pooling with the
    divisor folded forward, one member so the dense layer uses constants);
    with every 3x3 layer double-hoisted, and with a per-layer mix of single
    and double hoisting."""
    spec = nets.vgg_spec(seed=2, widths=(4, 4, 8, 8, 8), classes=5, image=(3, 16, 16), k=6, calib=4, hoist=hoist)
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print(f"[small_vgg] N=2^12 widths=(4,4,8,8,8) two pools hoist={hoist}", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 31)
    imgs = gen.images(14, 2, 3, 16, 16)
    gin = gnet.encrypt_images(keys, imgs, 900)
    gl = []
    gout, _ = gnet.run(keys, gin, hook=lambda ly, outs: gl.append((ly["name"], _coeff(ctx, outs[0]))))
    oin = onet.encrypt_image(sk, imgs[0], 900)
    ol = []
    oout, _ = onet.run(sk, oin, rlk, gk, hook=lambda ly, outs: ol.append((ly["name"], outs[0].data)))
    assert [n for n, _ in gl] == [n for n, _ in ol]
    for (n1, a), (n2, b) in zip(gl, ol):
        assert np.array_equal(a, b), n1
    from oracle.forward import forward
    for n in range(2):
        ref = forward(spec, imgs[n])
        got = gnet.decrypt_logits(keys, gout[n])
        assert np.max(np.abs(got - ref)) < 1e-3


@pytest.mark.parametrize("members", [1, 2])
def test_small_vgg_flattened_dense_bit_exact(members):
    """VGG-style network whose dense layer weighs every position of the
    flattened final map (ckc_layer_create_dense_spatial: the products with
    the K x C weight maps first, then the rotation sums of the K outputs):
    every layer bit-exact with the oracle, logits within 1e-3 of FP64; one
    and two members."""
    spec = nets.vgg_spec(seed=5, widths=(4, 4, 8, 8, 8), classes=5, image=(3, 16, 16), k=6, calib=4,
                         members=members, dense="flatten")
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print(f"[vgg_flatten] N=2^12 widths=(4,4,8,8,8) members={members} dense over the flattened 4x4 map", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 33)
    imgs = gen.images(16, 2, 3, 16, 16)
    gin = gnet.encrypt_images(keys, imgs, 950)
    gl = []
    gout, _ = gnet.run(keys, gin, hook=lambda ly, outs: gl.append((ly["name"], _coeff(ctx, outs[0]))))
    oin = onet.encrypt_image(sk, imgs[0], 950)
    ol = []
    oout, _ = onet.run(sk, oin, rlk, gk, hook=lambda ly, outs: ol.append((ly["name"], outs[0].data)))
    assert [n for n, _ in gl] == [n for n, _ in ol]
    for (n1, a), (n2, b) in zip(gl, ol):
        assert np.array_equal(a, b), n1
    from oracle.forward import forward
    for n in range(2):
        ref = forward(spec, imgs[n])
        got = gnet.decrypt_logits(keys, gout[n])
        assert np.max(np.abs(got - ref)) < 1e-3


def test_graphed_pass_replays_match_eager():
    """A network pass captured as a HIP graph and replayed for new inputs
    (eager work and synchronisations in between) gives the eager ciphertexts
    on every replay."""
    import torch
    from paper_2509_22857_amd.ckks import Context
    from paper_2509_22857_amd.graph import GraphedPass
    from paper_2509_22857_amd.network import GpuNetwork
    spec = nets.resnet_spec(seed=1, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16), k=8, calib=4)
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print("[graph] N=2^12 small resnet, 2 images per pass", flush=True)
    ctx = Context.from_params(ps)
    net = GpuNetwork(ctx, spec, D, D, D)
    keys = ctx.keygen(17, net.steps)
    gp = GraphedPass(net, keys, 2)
    for rep in range(3):
        imgs = gen.images(40 + rep, 2, 3, 16, 16)
        cts = net.encrypt_images(keys, imgs, 4096 * 8 * (rep + 1))
        eager, _ = net.run(keys, cts)
        torch.cuda.synchronize()
        want = [[c.buf.clone() for c in row] for row in eager]
        got = gp.run(cts)
        torch.cuda.synchronize()
        for wrow, grow in zip(want, got):
            for w, g in zip(wrow, grow):
                assert torch.equal(w, g.buf), rep


def test_native_runner_matches_python_orchestration():
    """The library's native runner (ckc_batch_plan / ckc_batch_run) executes
    the same layer program as the Python orchestration, bit for bit: a small
    ResNet ensemble (residual shortcuts, stride 2) and a small VGG (pooling;
    the dense after global average pooling, and over the flattened map),
    two requests under one key set batched together, a third under another
    key set in its own pass."""
    from paper_2509_22857_amd import ckks
    D = 2.0 ** 30
    cases = [
        ("resnet", nets.resnet_spec(seed=1, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16), k=8,
                                    calib=4), small_tower(logN=12, levels=6)),
        ("vgg", nets.vgg_spec(seed=2, widths=(4, 4, 8, 8, 8), classes=5, image=(3, 16, 16), k=6, calib=4),
         small_tower(logN=12, levels=6)),
        ("vgg_flatten", nets.vgg_spec(seed=2, widths=(4, 4, 8, 8, 8), classes=5, image=(3, 16, 16), k=6, calib=4,
                                      dense="flatten"), small_tower(logN=12, levels=6)),
    ]
    from paper_2509_22857_amd.ckks import Context
    from paper_2509_22857_amd.network import GpuNetwork
    for name, spec, ps in cases:
        print(f"[native] {name}", flush=True)
        ctx = Context.from_params(ps)
        gnet = GpuNetwork(ctx, spec, D, D, D)
        k1 = ctx.keygen(31, gnet.steps)
        k2 = ctx.keygen(32, gnet.steps)
        imgs = gen.images(77, 3, *spec["image"])
        ins = [gnet.encrypt_images(k, imgs[i:i + 1], 9000 + 64 * i)[0] for i, k in enumerate((k1, k1, k2))]
        want = [gnet.run(k, [row])[0][0] for k, row in zip((k1, k1, k2), ins)]
        plan = gnet.native_plan()
        assert plan.in_count == spec["image"][0] and plan.out_count == len(want[0])
        got = plan.run([k1, k1, k2], ins)
        for r in range(3):
            assert len(got[r]) == len(want[r])
            for a, b in zip(got[r], want[r]):
                assert a.level == b.level and a.scale == b.scale
                assert np.array_equal(_coeff(ctx, a), _coeff(ctx, b)), (name, r)
        with pytest.raises(ckks.CkcError, match="CKC_EINVAL"):
            ckks.Plan(ctx, '{"input": {"name": "x", "count": 3, "level": 0}, "output": "y", "steps": []}', [])


def test_slot_packed_images_bit_exact_and_accurate():
    """Two images packed into one set of ciphertexts (image p in member blocks
    p M .. p M + M - 1): every output ciphertext equals the oracle's on the
    same packed slots, and each image's logits match its own FP64 forward."""
    from oracle.ckks import Oracle
    from oracle.network import OracleNetwork
    from paper_2509_22857_amd.ckks import Context
    from paper_2509_22857_amd.network import GpuNetwork, packed_image_slots
    from oracle.forward import forward
    spec = nets.resnet_spec(seed=1, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16), k=8, calib=4)
    P, M = 2, 2
    pspec = nets.pack_spec(spec, P)
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print("[packed] 2 images x 2 members, N=2^12", flush=True)
    ctx = Context.from_params(ps)
    gnet = GpuNetwork(ctx, pspec, D, D, D)
    keys = ctx.keygen(41, gnet.steps)
    imgs = gen.images(88, P, *spec["image"])
    groups = gnet.encrypt_packed(keys, imgs, stream_base=3000)
    gout, _ = gnet.run(keys, groups)
    o = Oracle.from_params(ps)
    onet = OracleNetwork(o, pspec, D, D, D)
    sk = o.secret_key(41)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in onet.steps()}
    L = len(ps.q) - 1
    oin = [o.encrypt(o.encode(v, L, D), sk, 3000 + c) for c, v in enumerate(packed_image_slots(pspec, imgs, ps.N))]
    oout, _ = onet.run(sk, oin, rlk, gk)
    assert len(oout) == len(gout[0])
    for j, (g, w) in enumerate(zip(gout[0], oout)):
        assert np.array_equal(_coeff(ctx, g), w.data), j
    logits = gnet.decrypt_logits(keys, gout[0]).reshape(P, M, -1)
    for p in range(P):
        ref = forward(spec, imgs[p])
        assert np.max(np.abs(logits[p] - ref)) < 1e-3


def test_compiled_batch_normalised_network_bit_exact():
    """A trained-form network (batch normalisations, non-monic activations,
    projection and identity shortcuts, global average pooling) through the
    post-training compiler, then the evaluator: bit-exact with the oracle on
    the compiled description, logits within 1e-3 of its FP64 forward."""
    from oracle.forward import forward
    from paper_2509_22857_amd import compiler as cc
    from workloads.graphs import bn_resnet_graph
    g = bn_resnet_graph(seed=5, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16))
    spec, log = cc.compile_network(g, k=64, order="poly_first", direction="backward")
    assert {"case1", "case3", "case4"} <= {e[0] for e in log}
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print("[compiled_bn_resnet] N=2^12 M=2 widths=(4,8)", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 31)
    imgs = gen.images(60, 1, 3, 16, 16)
    gin = gnet.encrypt_images(keys, imgs, 700)
    gout, _ = gnet.run(keys, gin)
    oin = onet.encrypt_image(sk, imgs[0], 700)
    oout, _ = onet.run(sk, oin, rlk, gk)
    for k, (a, b) in enumerate(zip(gout[0], oout)):
        assert np.array_equal(_coeff(ctx, a), b.data), k
    got = gnet.decrypt_logits(keys, gout[0])
    assert np.max(np.abs(got - forward(spec, imgs[0]))) < 1e-3


def test_packed_logits_bit_exact():
    """The class ciphertexts of an image joined into one (mask, then a
    binary tree of rotations by -2^j): bit-exact with the oracle, class k of
    member m at slot m*block + k within 1e-3 of the FP64 forward."""
    spec = nets.resnet_spec(seed=1, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16), k=8, calib=4)
    spec["pack_output"] = True
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print("[packed_logits] N=2^12 M=2 classes=10", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 41)
    imgs = gen.images(19, 1, 3, 16, 16)
    gout, _ = gnet.run(keys, gnet.encrypt_images(keys, imgs, 1300))
    oout, _ = onet.run(sk, onet.encrypt_image(sk, imgs[0], 1300), rlk, gk)
    gp = gnet.pack_logits(keys, gout[0])
    op = onet.pack_logits(oout, gk)
    assert gp.level == op.level and gp.scale == op.scale
    assert np.array_equal(_coeff(ctx, gp), op.data)
    from oracle.forward import forward
    got = gnet.decrypt_packed_logits(keys, gp)
    assert np.max(np.abs(got - forward(spec, imgs[0]))) < 1e-3


def test_quantisation_aware_fitted_activation_network_bit_exact():
    """A network trained with the quantisation-aware ReLU fit of Section 3.2
    (d = 2, b = 10, c = 2: p(x) = (192 + 511 x + 240 x^2) / 2^10) at every
    activation, through the post-training compiler: bit-exact with the oracle,
    logits within 1e-3 of the FP64 forward of the compiled description."""
    from oracle.forward import forward
    from paper_2509_22857_amd import compiler as cc
    from paper_2509_22857_amd import qafit
    from workloads.graphs import bn_resnet_graph
    act = qafit.coefficients(2, 10, 2.0)
    assert tuple(np.round(act * 1024).astype(int)) == (192, 511, 240)
    g = bn_resnet_graph(seed=8, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16), act=act)
    spec, _ = cc.compile_network(g, k=64)
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print("[qafit_network] N=2^12 M=2 widths=(4,8), fitted activation", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 51)
    imgs = gen.images(61, 1, 3, 16, 16)
    gout, _ = gnet.run(keys, gnet.encrypt_images(keys, imgs, 800))
    oout, _ = onet.run(sk, onet.encrypt_image(sk, imgs[0], 800), rlk, gk)
    for k, (a, b) in enumerate(zip(gout[0], oout)):
        assert np.array_equal(_coeff(ctx, a), b.data), k
    got = gnet.decrypt_logits(keys, gout[0])
    ref = forward(spec, imgs[0])
    assert np.max(np.abs(got - ref)) < 1e-3
    assert got.mean(0).argmax() == ref.mean(0).argmax()


def test_slice_shared_resnet_bit_exact():
    """A ResNet-style ensemble in the slice-shared layout (blocks of 512 slots
    for 16x16 images: 16 spare rows): every layer bit-exact with the oracle,
    logits within 1e-3 of the FP64 forward; a third of the codebook
    plaintexts of the 3x3 layers."""
    spec = nets.resnet_spec(seed=1, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16), k=8, calib=4,
                            block_slots=512)
    spec["layout"]["slice_shared"] = True
    ps = small_tower(logN=12, levels=6)
    D = 2.0 ** 30
    print("[slice_shared_resnet] N=2^12 M=2 widths=(4,8) block 512", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 9)
    imgs = gen.images(3, 2, 3, 16, 16)
    gin = gnet.encrypt_images(keys, imgs, 100)
    gl = []
    gout, _ = gnet.run(keys, gin, hook=lambda ly, outs: gl.append((ly["name"], _coeff(ctx, outs[0]))))
    ol = []
    oout, _ = onet.run(sk, onet.encrypt_image(sk, imgs[0], 100), rlk, gk,
                       hook=lambda ly, outs: ol.append((ly["name"], outs[0].data)))
    for (n1, a), (n2, b) in zip(gl, ol):
        assert n1 == n2
        assert np.array_equal(a, b), n1
    from oracle.forward import forward
    for n in range(2):
        got = gnet.decrypt_logits(keys, gout[n])
        ref = forward(spec, imgs[n])
        assert np.max(np.abs(got - ref)) < 1e-3
    plain = dict(spec, layout=dict(spec["layout"], slice_shared=False))
    from paper_2509_22857_amd.network import GpuNetwork
    full = GpuNetwork(ctx, plain, D, D, D)
    for ly, e1, e2 in zip(spec["layers"], gnet.layers, full.layers):
        if ly["op"] == "conv" and ly["ksize"] == 3:
            assert e1["main"].nbytes() < 0.4 * e2["main"].nbytes(), ly["name"]


def test_tuned_hoisting_marks_bit_exact_and_replayed():
    """The per-layer key-switching form picked by timing both forms on the
    device (autotune.tune_hoisting) goes into the network description; the
    network with those marks is bit-exact with the oracle following the same
    marks, and a HIP-graph replay of a 2-image pass equals the eager pass."""
    import torch
    from paper_2509_22857_amd.autotune import tune_hoisting
    from paper_2509_22857_amd.graph import GraphedPass
    from paper_2509_22857_amd.network import GpuNetwork
    spec = nets.vgg_spec(seed=4, widths=(4, 8, 8), pool_after=(0,), classes=5, image=(3, 16, 16), k=6, calib=4)
    ps = small_tower(logN=12, levels=5)
    D = 2.0 ** 30
    print("[tuned_hoisting] N=2^12 small VGG", flush=True)
    ctx, gnet, keys, o, onet, sk, rlk, gk = _setup(ps, spec, D, D, D, 71)
    marks = tune_hoisting(gnet, keys, 2)
    assert len(marks) == sum(ly["op"] == "conv" for ly in spec["layers"])
    assert set(marks) <= {"single", "double"}
    nets.set_hoisting(spec, marks)
    gnet = GpuNetwork(ctx, spec, D, D, D)
    from oracle.network import OracleNetwork
    onet = OracleNetwork(o, spec, D, D, D)
    imgs = gen.images(72, 2, 3, 16, 16)
    gin = gnet.encrypt_images(keys, imgs, 1500)
    gout, _ = gnet.run(keys, gin)
    oout, _ = onet.run(sk, onet.encrypt_image(sk, imgs[0], 1500), rlk, gk)
    for j, (a, b) in enumerate(zip(gout[0], oout)):
        assert np.array_equal(_coeff(ctx, a), b.data), j
    torch.cuda.synchronize()
    want = [[c.buf.clone() for c in row] for row in gout]
    gp = GraphedPass(gnet, keys, 2)
    for rep in range(2):
        got = gp.run(gin)
        torch.cuda.synchronize()
        for wrow, grow in zip(want, got):
            for w, g in zip(wrow, grow):
                assert torch.equal(w, g.buf), rep
