"""GPU vs oracle, bit-exact, at the kernel instantiations the ResNet-20-style
ensemble runs: contraction workgroups of four images with double-buffered
codebook tiles, ragged image and output groups, extended key inner products
with 5 to 8 digits, and the grouped contraction of codebooks above 128
centroids.  Every case asserts, from the library's launch counts, that the
instantiation under test actually ran."""
import numpy as np
import pytest

from workloads import gen
from workloads.nets import single_conv_spec as _conv_spec
from workloads.params import small_tower

pytestmark = pytest.mark.gpu

D = 2.0 ** 30


@pytest.fixture(autouse=True)
def default_launch_choices():
    """The library's default launch choices (what the assertions on the
    instantiations taken assume), restored afterwards."""
    from paper_2509_22857_amd import ckks
    want = {"conv_outs": 8, "conv_imgs": 4, "ks_batch": 64, "conv_fuse": 1}
    saved = {k: ckks.tune_get(k) for k in want}
    for k, v in want.items():
        ckks.tune_set(k, v)
    yield
    for k, v in saved.items():
        ckks.tune_set(k, v)


def _run_both(ps, spec, n_img, seed):
    from oracle.ckks import Oracle
    from oracle.network import OracleNetwork
    from paper_2509_22857_amd import ckks
    from paper_2509_22857_amd.ckks import Context
    from paper_2509_22857_amd.network import GpuNetwork
    ctx = Context.from_params(ps)
    gnet = GpuNetwork(ctx, spec, D, D, D)
    keys = ctx.keygen(seed, gnet.steps)
    imgs = gen.images(seed + 1, n_img, *spec["image"])
    gin = gnet.encrypt_images(keys, imgs, 5000)
    ckks.variant_enable(True)
    try:
        gout, _ = gnet.run(keys, gin)
        counts = ckks.variant_counts()
    finally:
        ckks.variant_enable(False)
    o = Oracle.from_params(ps)
    onet = OracleNetwork(o, spec, D, D, D)
    sk = o.secret_key(seed)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in onet.steps()}
    # the first and last image of each 4-image contraction group (the GPU runs
    # them all; the oracle, slow at this size, checks these)
    for n in sorted({m for g0 in range(0, n_img, 4) for m in (g0, min(g0 + 3, n_img - 1))}):
        oin = onet.encrypt_image(sk, imgs[n], 5000 + n * 4096)
        oout, _ = onet.run(sk, oin, rlk, gk)
        assert len(oout) == len(gout[n])
        for j, (a, b) in enumerate(zip(gout[n], oout)):
            assert a.level == b.level and a.scale == b.scale, (n, j)
            assert np.array_equal(ctx.ct_to_coeff(a), b.data), (n, j)
    return counts


@pytest.mark.parametrize("levels", [4, 5, 6, 7])
def test_four_image_groups_and_high_digit_counts(levels):
    """One prime per digit, so a convolution at the top level of a chain of
    levels + 1 primes key-switches with levels + 1 = 5..8 digits; 7 images
    form a full 4-image workgroup and a ragged one of 3; 64 centroids, so the
    two codebook tiles of the double buffer fit; 12 outputs, so the second
    output group is ragged."""
    ps = small_tower(logN=12, levels=levels, alpha=1)
    dnum = levels + 1
    spec = _conv_spec(200 + levels, I=8, O=12, k=64, M=2)
    print(f"[variants] N=2^12 levels={levels} dnum={dnum} I=8 O=12 k=64, 7 images", flush=True)
    counts = _run_both(ps, spec, 7, 40 + levels)
    assert counts.get(f"kip_ext_rot<{dnum}>", 0) >= 1, counts
    assert counts.get("conv_mac<8,4>+dbuf+fused", 0) == 2, counts


def test_four_image_groups_without_double_buffer():
    """96 centroids: two codebook tiles no longer fit in 64 KiB, so the
    4-image workgroup stages one tile per tap; 5 images give a 4-image and
    a 1-image group."""
    ps = small_tower(logN=12, levels=3, alpha=2)
    spec = _conv_spec(301, I=6, O=9, k=96, M=2)
    print("[variants] N=2^12 k=96 I=6 O=9, 5 images", flush=True)
    counts = _run_both(ps, spec, 5, 61)
    assert counts.get("conv_mac<8,4>+fused", 0) == 1, counts
    assert counts.get("conv_mac<8,1>+fused", 0) == 1, counts


def test_grouped_contraction_above_128_centroids():
    """256 centroids per kernel column (the paper's larger codebooks): the
    grouped form runs (centroid groups summed before their one product)."""
    ps = small_tower(logN=12, levels=3, alpha=2)
    spec = _conv_spec(302, I=10, O=11, k=256, M=2)
    print("[variants] N=2^12 k=256 I=10 O=11 grouped, 2 images", flush=True)
    counts = _run_both(ps, spec, 2, 62)
    assert counts.get("conv_contract", 0) >= 1, counts
    assert not any(n.startswith("conv_mac") for n in counts), counts


def test_grouped_contraction_single_hoisted_stride_two():
    """The grouped form on a single-hoisted, stride-2 layer (rotated inputs
    back in Q_l, products over Q_l only)."""
    ps = small_tower(logN=12, levels=3, alpha=2)
    spec = _conv_spec(303, I=5, O=7, k=200, M=1, stride=2, hoist="single")
    print("[variants] N=2^12 k=200 single-hoisted stride 2", flush=True)
    counts = _run_both(ps, spec, 2, 63)
    assert counts.get("conv_contract", 0) >= 1, counts


def test_slice_shared_columns_four_image_groups():
    """Slice-shared layout (one codebook tile per kernel column, visited
    column by column; the P limbs skip the identity tap but keep its
    column's tile): 8 digits, 7 images in a double-buffered 4-image group and
    a ragged one, 16 spare rows under every 8x8 image."""
    ps = small_tower(logN=12, levels=7, alpha=1)
    spec = _conv_spec(211, I=8, O=12, k=64, M=2, block=128)
    spec["layout"]["slice_shared"] = True
    print("[variants] N=2^12 slice-shared dnum=8 I=8 O=12 k=64, 7 images", flush=True)
    counts = _run_both(ps, spec, 7, 48)
    assert counts.get("kip_ext_rot<8>", 0) >= 1, counts
    assert counts.get("conv_mac<8,4>+dbuf+fused", 0) == 2, counts


@pytest.mark.parametrize("hoist,k", [("double", 96), ("single", 200)])
def test_slice_shared_columns_other_forms(hoist, k):
    """Slice-shared layout with the single-buffered 4-image form (96
    centroids) and with the grouped form of a single-hoisted layer (200
    centroids), stride 2."""
    ps = small_tower(logN=12, levels=3, alpha=2)
    spec = _conv_spec(212, I=6, O=9, k=k, M=2, block=128, stride=2, hoist=hoist)
    spec["layout"]["slice_shared"] = True
    print(f"[variants] N=2^12 slice-shared {hoist} k={k} stride 2, 4 images", flush=True)
    counts = _run_both(ps, spec, 4, 64)
    if k <= 128:
        assert counts.get("conv_mac<8,4>+fused", 0) == 1, counts
    else:
        assert counts.get("conv_contract", 0) >= 1, counts


@pytest.mark.parametrize("layout,k,fuse", [("taps", 64, 1), ("slice", 64, 0), ("taps", 96, 1)])
def test_two_polynomials_per_contraction_wave(layout, k, fuse):
    """conv_rows = 2: each contraction wave takes both polynomials of its
    image (one codebook read from LDS per two products): double-buffered
    and single-buffered 4-image groups, a ragged 3-image group, the fused
    and the per-output-group launches, both layouts."""
    from paper_2509_22857_amd import ckks
    ps = small_tower(logN=12, levels=5, alpha=1)
    spec = _conv_spec(220 + k, I=8, O=12, k=k, M=2, block=128 if layout == "slice" else 64)
    spec["layout"]["slice_shared"] = layout == "slice"
    print(f"[variants] N=2^12 conv_rows=2 {layout} k={k} fuse={fuse}, 7 images", flush=True)
    ckks.tune_set("conv_rows", 2)
    ckks.tune_set("conv_fuse", fuse)
    try:
        counts = _run_both(ps, spec, 7, 70 + k)
    finally:
        ckks.tune_set("conv_rows", 1)
    dbuf = "+dbuf" if k <= 64 else ""
    if fuse:
        assert counts.get(f"conv_mac<8,4>{dbuf}+fused+rows2", 0) == 2, counts
    else:
        assert counts.get(f"conv_mac<8,4>{dbuf}+rows2", 0) >= 2, counts
    assert not any(n.startswith("conv_mac") and not n.endswith("rows2") for n in counts), counts
