"""Host logic of the CHW layout (no GPU): the slot vectors the product
builds for its plaintexts (diagonals rotated by their channel distance,
per-channel biases and activation coefficients, the packed input image) and
its rotation keys equal what the oracle's definition of the layout gives,
for full, repeated, widening and narrowing shapes; shapes outside the layout
are refused."""
import numpy as np
import pytest

from oracle.chw import OracleChw
from oracle.ckks import Oracle
from paper_2509_22857_amd.chw import ChwNetwork
from workloads.nets import chw_spec
from workloads.params import chw_chain


class _HostCtx:
    """What ChwNetwork reads from a context before any device call."""
    N = 4096
    q = list(chw_chain(12, 4).q)


@pytest.mark.parametrize("C,C1,C2,H,W", [(8, 8, 8, 16, 16), (32, 32, 32, 8, 8), (4, 4, 4, 16, 16),
                                         (4, 8, 2, 16, 16)])
def test_plaintext_slots_and_keys_match_the_oracle(C, C1, C2, H, W):
    spec = chw_spec(7, C=C, H=H, W=W, classes=4, C1=C1, C2=C2)
    net = ChwNetwork(_HostCtx(), spec, 2.0 ** 40)
    onet = OracleChw(Oracle.from_params(chw_chain(12, 4)), spec, 2.0 ** 40)
    for name in ("conv1_w", "conv2_w"):
        w = spec[name]
        for j in range(w.shape[1]):
            for t in range(9):
                want = np.roll(onet._diagonal(w, j, t // 3 - 1, t % 3 - 1), j * H * W)
                assert np.array_equal(np.roll(net._diag_slots(w, j, t), j * H * W), want), (name, j, t)
    for name in ("conv1_b", "act_b", "act_c", "conv2_b"):
        assert np.array_equal(net._per_block(spec[name]), onet._blocks(spec[name])), name
    assert net.steps == sorted(set(onet.steps()) - {0})
    img = np.random.default_rng(1).uniform(size=(C, H, W))
    z = np.tile(img.reshape(-1), 2048 // (C * H * W))
    assert np.array_equal(z, onet.slots_of(img))


def test_shapes_outside_the_layout_are_refused():
    with pytest.raises(ValueError):
        ChwNetwork(_HostCtx(), chw_spec(1, C=3, H=16, W=16), 2.0 ** 40)   # 3 channels
    with pytest.raises(ValueError):
        ChwNetwork(_HostCtx(), chw_spec(1, C=8, H=16, W=32), 2.0 ** 40)   # 8 x 512 > 2048 slots
    with pytest.raises(ValueError):
        ChwNetwork(_HostCtx(), chw_spec(1, C=4, H=12, W=12), 2.0 ** 40)   # 144-slot blocks
