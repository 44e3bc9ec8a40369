"""The oracle's slice-shared layout (one plaintext per kernel column and
centroid, vertical padding from zero rows; Section 5.2): it decrypts to the
FP64 convolution, leaves the spare rows at zero, needs those rows, and
carries through a whole ResNet-style network."""
import numpy as np
import pytest

from oracle.ckks import Oracle
from oracle.forward import forward
from oracle.network import OracleNetwork
from workloads import gen, nets
from workloads.params import small_tower

D = 2.0 ** 30


def _keys(o, net, seed):
    sk = o.secret_key(seed)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps()}
    return sk, rlk, gk


def _grid(z, B, W0, m, gap, H, W):
    return np.array([[z[m * B + gap * (r * W0 + c)] for c in range(W)] for r in range(H)])


def _one_conv(shared, block, stride=1):
    spec = nets.single_conv_spec(401, I=3, O=2, k=5, M=2, H=8, W=8, block=block, stride=stride)
    spec["layout"]["slice_shared"] = shared
    return spec


@pytest.mark.parametrize("stride", [1, 2])
def test_slice_shared_conv_decrypts_to_convolution_and_keeps_spare_rows_zero(stride):
    ps = small_tower(logN=12, levels=2)
    spec = _one_conv(True, 128, stride)  # 16 rows of 8: rows 8..15 of every block are spare
    o = Oracle.from_params(ps)
    net = OracleNetwork(o, spec, D, D, D)
    sk, rlk, gk = _keys(o, net, 3)
    img = gen.images(9, 1, 3, 8, 8)[0]
    outs, grid = net.run(sk, net.encrypt_image(sk, img, 10), rlk, gk)
    ref = forward(spec, img)  # [M][O][Ho][Wo]
    g, Ho, Wo = grid["gap"], grid["H"], grid["W"]
    for j, ct in enumerate(outs):
        z = o.decrypt_decode(ct, sk)
        for m in range(2):
            got = _grid(z, 128, 8, m, g, Ho, Wo)
            assert np.max(np.abs(got - ref[m, j])) < 2e-4, (m, j)
            # the spare rows of the block (base rows 8..15) hold zeros
            spare = z[m * 128 + 64:(m + 1) * 128]
            assert np.max(np.abs(spare)) < 2e-4, (m, j)


def test_slice_shared_layout_needs_spare_rows():
    """Without a zero row below the image the planner refuses the layout; with
    the check bypassed, the taps that leave the image at the top and bottom
    rows read the neighbouring member's pixels and the result is wrong there
    (and only there)."""
    ps = small_tower(logN=12, levels=2)
    spec = _one_conv(True, 64)  # 8 rows of 8: no spare row
    o = Oracle.from_params(ps)
    net = OracleNetwork(o, spec, D, D, D)
    sk, rlk, gk = _keys(o, net, 4)
    img = gen.images(10, 1, 3, 8, 8)[0]
    with pytest.raises(ValueError, match="rows per block"):
        net.run(sk, net.encrypt_image(sk, img, 20), rlk, gk)
    net._check_spare_rows = lambda grid: None
    outs, _ = net.run(sk, net.encrypt_image(sk, img, 20), rlk, gk)
    ref = forward(spec, img)
    z = o.decrypt_decode(outs[0], sk)
    got = _grid(z, 64, 8, 1, 1, 8, 8)
    err = np.abs(got - ref[1, 0])
    assert np.max(err[1:7]) < 2e-4
    assert np.max(err[[0, 7]]) > 1e-2


@pytest.mark.slow
def test_slice_shared_resnet_decrypts_to_forward():
    """A ResNet-style ensemble (stride-2 stage, projection shortcut,
    activations, global pooling and dense) in the slice-shared layout, blocks
    of 512 slots (32 rows of 16, the lower 16 spare): logits within 1e-3,
    same top-1."""
    spec = nets.resnet_spec(seed=1, members=2, widths=(4, 8), blocks=1, classes=10, image=(3, 16, 16), k=8, calib=4,
                            block_slots=512)
    spec["layout"]["slice_shared"] = True
    ps = small_tower(logN=12, levels=6)
    o = Oracle.from_params(ps)
    net = OracleNetwork(o, spec, D, D, D)
    sk, rlk, gk = _keys(o, net, 9)
    img = gen.images(3, 1, 3, 16, 16)[0]
    outs, _ = net.run(sk, net.encrypt_image(sk, img, 100), rlk, gk)
    got = np.array([[o.decrypt_decode(c, sk)[m * 512] for c in outs] for m in range(2)])
    ref = forward(spec, img)
    assert np.max(np.abs(got - ref)) < 1e-3
    assert got.mean(0).argmax() == ref.mean(0).argmax()
