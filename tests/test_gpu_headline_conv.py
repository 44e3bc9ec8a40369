"""One convolution layer of the ResNet-20-style ensemble at N = 2^16 on the
tower-reuse chain it runs on (level 20, 21 + 3 limbs, 7 digits, 4 members,
64 centroids, 4 images, double hoisting), in both layouts (one plaintext per
tap in 1024-slot blocks; slice-shared columns in 2048-slot blocks): every output
ciphertext is bit-identical to the oracle's, compared through the SHA-256
digests that tests/golden/make_headline_conv.py wrote from the oracle.  The
launch runs the instantiations the ensemble's step runs: a 4-image
contraction workgroup with double-buffered codebook tiles over both output
groups, and the 7-digit extended key inner product of the rotation group."""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


@pytest.mark.parametrize("name", ["headline_conv_N65536.json", "headline_conv_slice_N65536.json"])
def test_headline_conv_layer_matches_oracle_digests(name):
    from paper_2509_22857_amd import ckks
    from paper_2509_22857_amd.ckks import Context
    from paper_2509_22857_amd.network import GpuNetwork
    from workloads import gen
    from workloads.nets import single_conv_spec
    from workloads.params import resnet20_tower
    rec = json.load(open(os.path.join(GOLDEN, name)))
    c = rec["case"]
    ps = resnet20_tower()
    D = 2.0 ** rec["delta_log2"]
    spec = single_conv_spec(c["spec_seed"], c["I"], c["O"], c["k"], c["M"], c["H"], c["W"], c["block"])
    spec["layout"]["slice_shared"] = bool(c.get("slice_shared", False))
    print(f"[headline_conv] {name}: N=2^16 L=20 I={c['I']} O={c['O']} k={c['k']} M={c['M']} block={c['block']} "
          f"images={c['images']}", flush=True)
    ctx = Context.from_params(ps)
    net = GpuNetwork(ctx, spec, D, D, D)
    keys = ctx.keygen(c["key_seed"], net.steps)
    imgs = gen.images(c["image_seed"], c["images"], c["I"], c["H"], c["W"])
    gin = net.encrypt_images(keys, imgs, c["stream_base"])
    for n, row in enumerate(gin):
        got = [_digest(ctx.ct_to_coeff(x)) for x in row]
        assert got == rec["images"][n]["inputs"], f"input ciphertexts of image {n} differ"
    saved = {k: ckks.tune_get(k) for k in ("conv_outs", "conv_imgs", "conv_fuse")}
    ckks.tune_set("conv_outs", 8)
    ckks.tune_set("conv_imgs", 4)
    ckks.tune_set("conv_fuse", 1)
    ckks.variant_enable(True)
    try:
        gout, _ = net.run(keys, gin)
        counts = ckks.variant_counts()
    finally:
        ckks.variant_enable(False)
        for k, v in saved.items():
            ckks.tune_set(k, v)
    assert counts.get("conv_mac<8,4>+dbuf+fused", 0) == 1, counts
    assert counts.get("kip_ext_rot<7>", 0) >= 1, counts
    for n, row in enumerate(gout):
        want = rec["images"][n]["outputs"]
        assert len(row) == len(want)
        for j, (y, w) in enumerate(zip(row, want)):
            assert y.level == w["level"] and float(y.scale).hex() == w["scale"], (n, j)
            assert _digest(ctx.ct_to_coeff(y)) == w["sha256"], f"image {n} output {j}"
