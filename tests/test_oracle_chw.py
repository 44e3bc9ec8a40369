"""The CHW-layout network on the oracle (oracle/chw.py) against the float64
forward: the decrypted output of every stage (two 'same' convolutions in the
diagonal form over channels, the quadratic activation, sum pooling, the
dense layer) matches the forward's tensors, and the forward's convolution
matches scipy's 2-D correlation, also with the channel blocks repeated (4
channels of 16 x 16 fill half the slots, so two copies) and with convolutions
that widen and narrow the channels (4 -> 8 -> 2).  A diagonal taken the wrong
way round (input channel o - d instead of o + d) is caught."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle.chw import OracleChw
from oracle.ckks import Oracle
from oracle.forward import _conv, forward_chw
from workloads import gen
from workloads.nets import chw_spec
from workloads.params import chw_chain


def test_forward_conv_is_scipy_correlation():
    g = np.random.default_rng(3)
    x = g.normal(size=(5, 7, 6))
    w = g.normal(size=(4, 5, 3, 3))
    b = g.normal(size=4)
    want = np.stack([sum(correlate2d(x[i], w[o, i], mode="same") for i in range(5)) + b[o] for o in range(4)])
    assert np.allclose(_conv(x, w, b, 1), want, atol=1e-12)


def _setup(C, H, W, C1=None, C2=None, seed=5):
    ps = chw_chain(12, 4)
    spec = chw_spec(seed, C=C, H=H, W=W, classes=4, C1=C1, C2=C2)
    o = Oracle.from_params(ps)
    net = OracleChw(o, spec, 2.0 ** ps.delta_log2)
    sk = o.secret_key(11)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps() if o.galois_elt(s) != 1}
    img = gen.images(12, 1, C, H, W)[0]
    return o, spec, net, sk, gk, img


@pytest.mark.parametrize("C,C1,C2,H,W", [(8, 8, 8, 16, 16), (2, 2, 2, 32, 32), (4, 4, 4, 16, 16),
                                         (4, 8, 2, 16, 16)])
def test_chw_network_decrypts_to_the_forward(C, C1, C2, H, W):
    o, spec, net, sk, gk, img = _setup(C, H, W, C1, C2)
    out = net.run(net.encrypt_image(sk, img, 100), o.relin_key(sk), gk)
    cap = {}
    logits = forward_chw(spec, img, cap)
    for name, ch in (("conv1", C1), ("act", C1), ("conv2", C2)):
        got = net.grid_of(o.decrypt_decode(out[name], sk), ch)
        assert np.max(np.abs(got - cap[name])) < 1e-6, name
    pool = o.decrypt_decode(out["pool"], sk)[np.arange(C2) * H * W]
    assert np.max(np.abs(pool - cap["pool"])) < 1e-5
    got = np.array([o.decrypt_decode(c, sk)[0] for c in out["logits"]])
    assert np.max(np.abs(got - logits)) < 1e-6
    assert [c.level for c in out["logits"]] == [0] * 4


def test_a_diagonal_the_wrong_way_round_is_caught():
    o, spec, net, sk, gk, img = _setup(8, 16, 16)
    right = net._diagonal

    def wrong(w, d, dh, dw):
        return right(w, (-d) % w.shape[1], dh, dw)

    net._diagonal = wrong
    y = net.conv(net.encrypt_image(sk, img, 100), spec["conv1_w"], spec["conv1_b"], gk)
    cap = {}
    forward_chw(spec, img, cap)
    assert np.max(np.abs(net.grid_of(o.decrypt_decode(y, sk), 8) - cap["conv1"])) > 0.1
