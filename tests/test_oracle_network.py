"""Oracle network evaluation against the FP64 forward, the generator's
independent forward, and the paper's level counts."""
import numpy as np
import pytest

from oracle.ckks import Oracle
from oracle.forward import forward
from oracle.network import OracleNetwork
from workloads import gen
from workloads import nets
from workloads.params import tiny, small_tower, resnet20_tower


def test_forward_matches_generator_forward():
    """Two independent numpy paths of the same network agree (calibration
    forward of the generator vs the oracle's forward)."""
    spec = nets.resnet_spec(seed=3, members=2, widths=(4, 8), blocks=1, classes=5, image=(3, 8, 8), k=6, calib=2)
    img = gen.images(11, 1, 3, 8, 8)[0]
    ref = forward(spec, img)
    M = spec["members"]
    t = {"x": np.broadcast_to(img[None, None], (M, 1) + img.shape).copy()}
    for ly in spec["layers"]:
        x = t[ly["inp"]]
        if ly["op"] == "conv":
            y = nets._conv_fwd(x, nets.conv_weights(ly["codebook"], ly["idx"]), ly["bias"], ly["stride"])
            if ly.get("short"):
                sh = ly["short"]
                y = y + nets._conv_fwd(t[sh["inp"]], nets.conv_weights(sh["codebook"], sh["idx"]), None, sh["stride"])
        elif ly["op"] == "act":
            y = ly["a_absorb"] * (x * x + ly["b"][:, None, :, None, None] * x + ly["c"][:, None, :, None, None])
        elif ly["op"] == "dense":
            y = np.einsum("mbc,mkc->mbk", x.sum(axis=(3, 4)), ly["w"]) + ly["bias"][:, None, :]
        t[ly["out"]] = y
    assert np.allclose(t["logits"][:, 0], ref, rtol=1e-12, atol=1e-12)


def test_clustering_respects_slices():
    spec = nets.resnet_spec(seed=4, members=3, widths=(4,), blocks=1, classes=3, image=(3, 8, 8), k=5, calib=2)
    for ly in spec["layers"]:
        if ly["op"] == "conv":
            assert ly["codebook"].shape[1] == 5 and ly["codebook"].shape[2] == 3
            assert ly["idx"].max() < 5
            W = nets.conv_weights(ly["codebook"], ly["idx"])
            # one codebook per kernel column: each column uses at most k distinct member vectors
            for col in range(ly["ksize"]):
                rows = W[:, :, :, :, col].reshape(3, -1).T
                assert len(np.unique(rows, axis=0)) <= 5


def test_kmeans_recovers_separated_clusters():
    g = gen.rng(0)
    centres = np.array([[-1.0, 0.5], [0.0, 0.0], [2.0, -1.0]])
    X = np.concatenate([c + 0.01 * g.standard_normal((50, 2)) for c in centres])
    C, lab = nets.kmeans_rows(X, 3)
    got = C[np.argsort(C[:, 0])]
    assert np.allclose(got, centres[np.argsort(centres[:, 0])], atol=0.01)
    assert len(set(lab[:50])) == 1 and len(set(lab[50:100])) == 1


def test_tiny_network_decrypts_to_forward():
    ps = tiny()
    spec = nets.tiny_spec(0)
    o = Oracle.from_params(ps)
    net = OracleNetwork(o, spec, delta=2.0 ** 40, target=2.0 ** 34, in_scale=2.0 ** 40)
    sk = o.secret_key(7)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps()}
    img = gen.images(5, 1, 1, 8, 8)[0]
    outs, grid = net.run(sk, net.encrypt_image(sk, img, 100), rlk, gk)
    assert outs[0].level == 0
    z = o.decrypt_decode(outs[0], sk)
    got = np.array([[z[grid["gap"] * (r * 8 + c)] for c in range(8)] for r in range(8)])
    ref = forward(spec, img)[0, 0]
    assert np.max(np.abs(got - ref)) < 1e-5


def test_activation_and_dense_network_decrypts_to_forward():
    """The activation + pooled dense network of the headline act/dense digest
    case, at N = 2^12: the oracle's logits (slot m B of each class
    ciphertext) are the FP64 forward's."""
    spec = nets.act_dense_spec(11, C=4, M=2, classes=3, H=8, W=8, block=64)
    ps = small_tower(logN=12, levels=4)
    o = Oracle.from_params(ps)
    D = 2.0 ** 30
    net = OracleNetwork(o, spec, delta=D, target=D, in_scale=D)
    sk = o.secret_key(12)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps()}
    img = gen.images(13, 1, 4, 8, 8)[0]
    outs, _ = net.run(sk, net.encrypt_image(sk, img, 100), rlk, gk)
    got = np.array([[o.decrypt_decode(c, sk)[m * 64] for c in outs] for m in range(2)])
    ref = forward(spec, img)
    # the network written out: per member m, class k: the sum over channels
    # and pixels of w[m][k][c] (x^2 + b x + c), plus the bias
    act = img[None] ** 2 + spec["layers"][0]["b"][:, :, None, None] * img[None] + \
        spec["layers"][0]["c"][:, :, None, None]
    direct = np.einsum("mkc,mc->mk", spec["layers"][1]["w"], act.sum(axis=(2, 3))) + spec["layers"][1]["bias"]
    assert ref.shape == (2, 3) and np.allclose(ref, direct, rtol=0, atol=1e-12)
    assert np.max(np.abs(got - ref)) < 1e-4


def test_flattened_dense_network_decrypts_to_forward():
    """A VGG-style network whose dense layer weighs every position of the
    flattened final map (the products first, then the slot sums over the
    grid): the oracle's logits are the FP64 forward's, and the forward's
    dense is the dot product with the flattened map, written out."""
    spec = nets.vgg_spec(seed=3, widths=(4, 6), pool_after=(0,), classes=3, image=(3, 8, 8), k=6, calib=4,
                         dense="flatten")
    assert np.shape(spec["layers"][-1]["w"]) == (1, 3, 6, 4, 4)
    ps = small_tower(logN=12, levels=6)
    o = Oracle.from_params(ps)
    D = 2.0 ** 30
    net = OracleNetwork(o, spec, delta=D, target=D, in_scale=D)
    sk = o.secret_key(14)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps()}
    img = gen.images(15, 1, 3, 8, 8)[0]
    outs, _ = net.run(sk, net.encrypt_image(sk, img, 100), rlk, gk)
    got = np.array([[o.decrypt_decode(c, sk)[0] for c in outs]])
    cap = {}
    ref = forward(spec, img, capture=cap)
    fc = spec["layers"][-1]
    fmap = cap[fc["inp"]][0]
    assert np.allclose(ref[0], np.einsum("kchw,chw->k", fc["w"][0], fmap) + fc["bias"][0], rtol=0, atol=1e-12)
    assert np.max(np.abs(got - ref)) < 1e-4


@pytest.mark.slow
def test_small_resnet_ensemble_decrypts_to_forward():
    spec = nets.resnet_spec(seed=1, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16), k=8, calib=4)
    ps = small_tower(logN=12, levels=6)
    o = Oracle.from_params(ps)
    D = 2.0 ** 30
    net = OracleNetwork(o, spec, delta=D, target=D, in_scale=D)
    sk = o.secret_key(9)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps()}
    img = gen.images(3, 1, 3, 16, 16)[0]
    outs, _ = net.run(sk, net.encrypt_image(sk, img, 100), rlk, gk)
    assert outs[0].level == 0
    B = spec["layout"]["block"]
    got = np.array([[o.decrypt_decode(c, sk)[m * B] for c in outs] for m in range(2)])
    ref = forward(spec, img)
    assert np.max(np.abs(got - ref)) < 1e-3
    assert got.mean(0).argmax() == ref.mean(0).argmax()


def _count_levels(spec, ps, delta):
    from paper_2509_22857_amd.network import plan_network
    plans, state = plan_network(spec, ps.q, delta, delta, delta)
    return len(ps.q) - 1 - state[spec["layers"][-1]["out"]][0], sum(p.rescale for p in plans)


def test_tower_reuse_level_count_resnet20():
    """Section 4.4 (levels table): ResNet-20 needs 20 levels with every
    optimisation (tower reuse halves the per-layer count)."""
    spec = nets.resnet_spec(seed=0, members=1, widths=(16, 32, 64), blocks=3, classes=10, image=(3, 32, 32), k=4,
                            calib=1)
    ps = resnet20_tower()
    used, rescales = _count_levels(spec, ps, 2.0 ** 30)
    assert used == 20 and rescales == 20


@pytest.mark.parametrize("widths,blocks,levels", [((64, 128, 256, 512), 2, 18), ((16, 32, 64), 5, 32)])
def test_tower_reuse_level_counts_resnet18_resnet32(widths, blocks, levels):
    """Section 4.4's level table: ResNet-18 needs 18 levels and ResNet-32 32
    with node fusing, weight redistribution and tower reuse."""
    spec = nets.resnet_spec(seed=0, members=1, widths=widths, blocks=blocks, classes=10, image=(3, 32, 32), k=4,
                            calib=1)
    used, _ = _count_levels(spec, resnet20_tower(levels=levels + 2), 2.0 ** 30)
    assert used == levels


def test_tower_reuse_halves_the_levels_resnet20():
    """Section 4.4's law: with tower reuse the level count is ceil(L / 2) of
    the count without it.  ResNet-20 on a chain of primes ~ Delta (every
    multiplicative layer rescales) uses 39 levels; on q_i ~ Delta^2, 20."""
    from workloads.params import balanced_chain, nearest_prime
    spec = nets.resnet_spec(seed=0, members=1, widths=(16, 32, 64), blocks=3, classes=10, image=(3, 32, 32), k=4,
                            calib=1)
    two_n = 2 << 16
    q = balanced_chain([30] * 48, two_n)
    q = [nearest_prime(40, two_n, exclude=q)] + q
    from paper_2509_22857_amd.network import plan_network
    D = 2.0 ** 30
    plans, state = plan_network(spec, q, D, D, D)
    std = len(q) - 1 - state[spec["layers"][-1]["out"]][0]
    tower, _ = _count_levels(spec, resnet20_tower(), D)
    assert std == 39 and tower == 20 == -(-std // 2)


def test_standard_chain_rescales_after_every_product():
    """With every prime ~ Delta (sublevel 1) the rule degenerates to the
    standard chain: one rescale per multiplicative layer (the tiny case)."""
    ps = tiny()
    spec = nets.tiny_spec(0)
    from paper_2509_22857_amd.network import plan_network
    plans, state = plan_network(spec, ps.q, 2.0 ** 40, 2.0 ** 34, 2.0 ** 40)
    assert [p.rescale for p in plans] == [True, True]
    assert state["y"][0] == 0


def test_planner_rejects_chains_without_headroom():
    """A chain whose last prime cannot hold the activation's squared scale
    (Delta^2 ~ q_0) is refused instead of wrapping the message."""
    from paper_2509_22857_amd.network import plan_network
    from workloads.params import small_tower
    spec = nets.vgg_spec(seed=2, widths=(4, 4, 8, 8, 8), classes=5, image=(3, 16, 16), k=6, calib=4)
    with pytest.raises(ValueError):
        plan_network(spec, small_tower(logN=12, levels=4).q, 2.0 ** 30, 2.0 ** 30, 2.0 ** 30)
    plans, state = plan_network(spec, small_tower(logN=12, levels=6).q, 2.0 ** 30, 2.0 ** 30, 2.0 ** 30)
    assert min(p.level for p in plans) >= 1


def test_pack_spec_repeats_members_per_image():
    """Slot packing changes no arithmetic: with the same image in every group
    of member blocks, the packed network's logits are the original network's
    logits repeated once per packed image."""
    spec = nets.resnet_spec(seed=6, members=2, widths=(4, 8), blocks=1, classes=5, image=(3, 8, 8), k=6, calib=2)
    packed = nets.pack_spec(spec, 3)
    assert packed["members"] == 6 and packed["packed"] == {"images": 3, "members": 2}
    img = gen.images(21, 1, 3, 8, 8)[0]
    assert np.allclose(forward(packed, img), np.tile(forward(spec, img), (3, 1)), rtol=1e-12, atol=1e-12)


def test_single_hoisted_convolutions_decrypt_to_forward():
    """Both key-switching forms of a 3x3 layer (one ModDown per output, or
    one per rotated input) decrypt to the FP64 forward; their ciphertexts
    differ in the low bits (the ModDowns round at different places)."""
    ps = small_tower(logN=12, levels=4)
    o = Oracle.from_params(ps)
    D = 2.0 ** 30
    img = gen.images(4, 1, 3, 8, 8)[0]
    sk = o.secret_key(13)
    rlk = o.relin_key(sk)
    got = {}
    for mode in ("single", "double"):
        spec = nets.vgg_spec(seed=2, widths=(4, 4), pool_after=(0,), classes=3, image=(3, 8, 8), k=4, calib=2,
                             hoist=mode)
        net = OracleNetwork(o, spec, delta=D, target=D, in_scale=D)
        gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps()}
        outs, _ = net.run(sk, net.encrypt_image(sk, img, 100), rlk, gk)
        got[mode] = outs
        vals = np.array([o.decrypt_decode(c, sk)[0] for c in outs])
        assert np.max(np.abs(vals - forward(spec, img)[0])) < 1e-3
    assert any(not np.array_equal(a.data, b.data) for a, b in zip(got["single"], got["double"]))
    with pytest.raises(ValueError):
        nets.vgg_spec(seed=2, widths=(4, 4), pool_after=(0,), classes=3, image=(3, 8, 8), k=4, calib=2,
                      hoist=["single"])


def test_hoisting_choice_of_the_benchmarked_networks():
    """The operation-count choice of key-switching form: every ResNet-20 3x3
    layer double-hoisted; the VGG-style network single-hoisted at its first
    layer (3 inputs, 64 outputs: more outputs than rotated inputs) and at
    its last (level 2: three Q limbs plus three P limbs), as bench.py runs
    it."""
    import bench
    from paper_2509_22857_amd.network import choose_hoisting
    ps = resnet20_tower(levels=6)
    D = 2.0 ** ps.delta_log2
    spec = nets.vgg_spec(seed=0, calib=2)
    assert choose_hoisting(spec, ps.q, len(ps.p), D, D, D) == bench.VGG_HOISTING
    ps = resnet20_tower()
    D = 2.0 ** ps.delta_log2
    spec = nets.resnet_spec(seed=0, members=4, widths=(16, 32, 64), blocks=3, classes=100, image=(3, 32, 32),
                            k=64, calib=2)
    assert set(choose_hoisting(spec, ps.q, len(ps.p), D, D, D)) == {"double"}


def test_packed_logits_decrypt_to_forward():
    """The class ciphertexts joined into one (mask of the slots m*block, then
    a binary tree of rotations by -2^j): class k of member m decrypts at slot
    m*block + k to the FP64 forward, with the same precision as unpacked."""
    ps = small_tower(logN=12, levels=4)
    o = Oracle.from_params(ps)
    D = 2.0 ** 30
    spec = nets.vgg_spec(seed=2, widths=(4, 4), pool_after=(0,), classes=5, image=(3, 8, 8), k=4, calib=2)
    spec["pack_output"] = True
    net = OracleNetwork(o, spec, delta=D, target=D, in_scale=D)
    assert {-1, -2, -4} <= set(net.steps())
    sk = o.secret_key(17)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps()}
    img = gen.images(6, 1, 3, 8, 8)[0]
    outs, _ = net.run(sk, net.encrypt_image(sk, img, 100), rlk, gk)
    packed = net.pack_logits(outs, gk)
    z = o.decrypt_decode(packed, sk)
    B = spec["layout"]["block"]
    ref = forward(spec, img)
    got = np.array([[z[m * B + k] for k in range(5)] for m in range(spec["members"])])
    assert np.max(np.abs(got - ref)) < 1e-3
    # every other slot of a member's block holds (nearly) zero
    assert np.max(np.abs(z[5:B])) < 1e-3


def test_tower_reuse_worked_example():
    """Section 4.3's example: with q_i ~ Delta^2 (sublevel 2), an input at
    sublevel 1 squared by the activation stays at sublevel 2 (no rescale); the
    next convolution with weights at sublevel 1 reaches sublevel 3 > 2, so it
    rescales, and the result is back at sublevel 1."""
    from paper_2509_22857_amd.network import plan_network, sublevel
    spec = nets.vgg_spec(seed=1, widths=(4, 4), pool_after=(), classes=2, image=(3, 8, 8), k=4, calib=1)
    ps = resnet20_tower(levels=4)
    D = 2.0 ** 30
    plans, state = plan_network(spec, ps.q, D, D, D)
    conv0, act0, conv1, act1 = plans[:4]
    assert sublevel(float(ps.q[conv1.level]), D) == 2
    assert sublevel(act0.in_scale, D) == 1 and not act0.rescale and sublevel(act0.out_scale, D) == 2
    assert sublevel(conv1.in_scale, D) == 2 and sublevel(conv1.pt_scale, D) == 1
    assert sublevel(conv1.out_scale, D) == 3 and conv1.rescale
    assert sublevel(conv1.out_scale / float(ps.q[conv1.level]), D) == 1
