"""The CHW layout on the GPU (paper_2509_22857_amd/chw.py: every channel of
an image in one ciphertext, convolutions in the diagonal form over channels,
evaluated baby-step giant-step: one hoisted group of the 9 tap rotations,
one 9-term plaintext MAC and one rotation per channel distance) against the
oracle's definition of the same network (oracle/chw.py): the input and every
stage's output ciphertext bit-identical, with equal levels and scales, and
the decrypted logits within 1e-6 of the float64 forward.  Shapes: 8 channels
of 16 x 16 and 32 channels of 8 x 8 fill the 2048 slots of N = 2^12; 4
channels of 16 x 16 fill half of them, repeated twice; and convolutions that
widen and narrow the channels (4 -> 8 -> 2)."""
import numpy as np
import pytest

from workloads import gen
from workloads.nets import chw_spec
from workloads.params import chw_chain

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("C,C1,C2,H,W", [(8, 8, 8, 16, 16), (32, 32, 32, 8, 8), (4, 4, 4, 16, 16), (4, 8, 2, 16, 16)])
def test_chw_network_bit_exact_with_oracle(C, C1, C2, H, W):
    from oracle.chw import OracleChw
    from oracle.ckks import Oracle
    from oracle.forward import forward_chw
    from paper_2509_22857_amd.chw import ChwNetwork
    from paper_2509_22857_amd.ckks import Context
    ps = chw_chain(12, 4)
    D = 2.0 ** ps.delta_log2
    spec = chw_spec(7, C=C, H=H, W=W, classes=4, C1=C1, C2=C2)
    print(f"[chw] N=2^12 channels {C}-{C1}-{C2} H={H} W={W}", flush=True)
    ctx = Context.from_params(ps)
    net = ChwNetwork(ctx, spec, D)
    keys = ctx.keygen(21, net.steps)
    img = gen.images(22, 1, C, H, W)[0]
    x = net.encrypt_image(keys, img, 300)
    out = net.run(keys, x)

    o = Oracle.from_params(ps)
    onet = OracleChw(o, spec, D)
    sk = o.secret_key(21)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in onet.steps() if o.galois_elt(s) != 1}
    ox = onet.encrypt_image(sk, img, 300)
    assert np.array_equal(ctx.ct_to_coeff(x), ox.data)
    oout = onet.run(ox, o.relin_key(sk), gk)
    for name in ("conv1", "act", "conv2", "pool"):
        a, b = out[name], oout[name]
        assert a.level == b.level and a.scale == b.scale, name
        assert np.array_equal(ctx.ct_to_coeff(a), b.data), name
    for k, (a, b) in enumerate(zip(out["logits"], oout["logits"])):
        assert a.level == b.level == 0 and a.scale == b.scale, k
        assert np.array_equal(ctx.ct_to_coeff(a), b.data), k
    got = net.decrypt_logits(keys, out["logits"])
    assert np.max(np.abs(got - forward_chw(spec, img))) < 1e-6
