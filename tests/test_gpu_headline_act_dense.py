"""The activation and the dense layer of a ResNet-20-style ensemble at
N = 2^16 on the tower-reuse chain it runs on: a monic quadratic activation
of 16 channels of 32x32 with relinearisation at the top level (7
key-switching digits), then the dense layer after global sum pooling (slot
sums by rotation, 10 classes) over 4 members.  Every output ciphertext is
bit-identical to the oracle's, compared through the SHA-256 digests that
tests/golden/make_headline_act_dense.py wrote from the oracle, and the
decrypted logits are within 1e-3 of the FP64 forward."""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "headline_act_dense_N65536.json")


def _digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def test_headline_act_and_dense_match_oracle_digests():
    from oracle.forward import forward
    from paper_2509_22857_amd import ckks
    from paper_2509_22857_amd.ckks import Context
    from paper_2509_22857_amd.network import GpuNetwork
    from workloads import gen
    from workloads.nets import act_dense_spec
    from workloads.params import resnet20_tower
    rec = json.load(open(GOLDEN))
    c = rec["case"]
    ps = resnet20_tower()
    D = 2.0 ** rec["delta_log2"]
    spec = act_dense_spec(c["spec_seed"], c["C"], c["M"], c["classes"], c["H"], c["W"], c["block"])
    print(f"[headline_act_dense] N=2^16 L=20 C={c['C']} M={c['M']} classes={c['classes']} images={c['images']}",
          flush=True)
    ctx = Context.from_params(ps)
    net = GpuNetwork(ctx, spec, D, D, D)
    keys = ctx.keygen(c["key_seed"], net.steps)
    imgs = gen.images(c["image_seed"], c["images"], c["C"], c["H"], c["W"])
    gin = net.encrypt_images(keys, imgs, c["stream_base"])
    for n, row in enumerate(gin):
        assert [_digest(ctx.ct_to_coeff(x)) for x in row] == rec["images"][n]["inputs"], n
    ckks.variant_enable(True)
    try:
        gout, _ = net.run(keys, gin)
        counts = ckks.variant_counts()
    finally:
        ckks.variant_enable(False)
    assert counts.get("kip_b<7>", 0) >= 1, counts
    for n, row in enumerate(gout):
        want = rec["images"][n]["outputs"]
        assert len(row) == len(want)
        for j, (y, w) in enumerate(zip(row, want)):
            assert y.level == w["level"] and float(y.scale).hex() == w["scale"], (n, j)
            assert _digest(ctx.ct_to_coeff(y)) == w["sha256"], f"image {n} output {j}"
        err = np.max(np.abs(net.decrypt_logits(keys, row) - forward(spec, imgs[n])))
        assert err < 1e-3, (n, err)
