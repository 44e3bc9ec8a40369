"""Post-training compiler (node fusing, weight redistribution, slice-ensemble
clustering, lowering): every pass leaves the network's function unchanged.

Pins: the fused coefficients of Cases 1-4 against the composed functions
evaluated directly; the redistribution updates against the defining
equalities (leading coefficient 1, function unchanged, backward update
c_d^(1/d) in the producer); whole compiled networks, run by the oracle's
forward of the evaluator's description, against the oracle's forward of the
original graph with batch normalisations (two independent interpreters)."""
import numpy as np
import pytest

from oracle import graph as og
from oracle.forward import forward as spec_forward
from paper_2509_22857_amd import compiler as cc
from workloads import gen
from workloads.graphs import bn_resnet_graph, bn_vgg_graph


def _close(a, b, rel=1e-12):
    assert np.max(np.abs(a - b)) <= rel * max(1.0, float(np.max(np.abs(b)))), np.max(np.abs(a - b))


def _rand(r, *shape):
    return r.uniform(-1.5, 1.5, shape)


def test_node_fusing_closed_forms_match_composition():
    r = np.random.default_rng(1)
    n = 50
    b1, b0, bx1, bx0, by1, by0 = (_rand(r, n) for _ in range(6))
    c = _rand(r, n, 3)
    x, y = _rand(r, n), _rand(r, n)

    def P(z):
        return c[:, 2] * z * z + c[:, 1] * z + c[:, 0]

    # Case 1: P(B(x)) is the fused quadratic
    p = cc.fuse_case1(b1, b0, c)
    _close(p[:, 2] * x * x + p[:, 1] * x + p[:, 0], P(b1 * x + b0))

    def S(d, x, y):
        return sum(d[:, i, j] * x ** i * y ** j for i in range(3) for j in range(3 - i))

    # Case 3: P(B_X(x) + B_Y(y)); Case 4: P(B_X(x) + y)
    _close(S(cc.fuse_case3(bx1, bx0, by1, by0, c), x, y), P(bx1 * x + bx0 + by1 * y + by0))
    _close(S(cc.fuse_case4(bx1, bx0, c), x, y), P(bx1 * x + bx0 + y))
    # Case 2: B(K(x)) for a kernel K(x) = sum_i w_i x_i + beta (per output channel)
    W, beta, v = _rand(r, 1, n, 7), _rand(r, 1, n), _rand(r, 7)
    Wf, af = cc.fuse_case2(b1[None], b0[None], W, beta)
    _close(Wf[0] @ v + af[0], b1 * (W[0] @ v + beta[0]) + b0)
    Wf, af = cc.fuse_case2(b1[None], b0[None], W, None)
    _close(Wf[0] @ v + af[0], b1 * (W[0] @ v) + b0)


def _chain(M, C, first, second):
    """x -> first -> second on a C-channel 4x4 grid."""
    return dict(members=M, image=(C, 4, 4), nodes=[dict(first, inp=["x"], out="a"), dict(second, inp=["a"], out="b")])


def _poly(r, M, C, d=2, positive=True):
    c = _rand(r, M, C, d + 1)
    if positive:
        c[..., -1] = r.uniform(0.1, 2.0, (M, C))
    return dict(op="poly", name="p", c=c)


def _bn(r, M, C):
    return dict(op="bn", name="bn", gamma=_rand(r, M, C), beta=_rand(r, M, C), mean=_rand(r, M, C),
                var=r.uniform(0.5, 2.0, (M, C)), eps=1e-5)


def _conv(r, M, C, k=3):
    return dict(op="conv", name="k", W=_rand(r, M, C, C, k, k), b=_rand(r, M, C), stride=1)


@pytest.mark.parametrize("direction", ["forward", "backward"])
def test_redistribution_identities(direction):
    r = np.random.default_rng(2)
    M, C = 2, 3
    img = _rand(r, C, 4, 4)
    cases = {
        "poly->conv": _chain(M, C, _poly(r, M, C), _conv(r, M, C)),
        "conv->poly": _chain(M, C, _conv(r, M, C), _poly(r, M, C)),
        "poly->poly": _chain(M, C, _poly(r, M, C), dict(_poly(r, M, C, 3), name="q")),
        "conv->cubic": _chain(M, C, _conv(r, M, C), _poly(r, M, C, 3, positive=False)),
        "poly->bn": _chain(M, C, _poly(r, M, C), _bn(r, M, C)),
        "bn->poly": _chain(M, C, _bn(r, M, C), _poly(r, M, C)),
    }
    bi = dict(members=M, image=(C, 4, 4), nodes=[
        dict(_conv(r, M, C), name="k1", inp=["x"], out="a"),
        dict(_conv(r, M, C, 1), name="k2", inp=["x"], out="b"),
        dict(op="bipoly", name="s", inp=["a", "b"], out="s", c=_rand(r, M, C, 3, 3)),
        dict(_conv(r, M, C), name="k3", inp=["s"], out="o")])
    bi["nodes"][2]["c"][..., 2, 0] = r.uniform(0.1, 2.0, (M, C))
    cases["bipoly"] = bi
    for name, g in cases.items():
        ref = og.forward(g, img)
        out, log = cc.redistribute(g, direction)
        _close(og.forward(out, img), ref, 1e-11)
        for n in out["nodes"]:
            if n["op"] == "poly":
                assert np.all(n["c"][..., -1] == 1.0), name
            if n["op"] == "bipoly":
                assert np.all(n["c"][..., 2, 0] == 1.0), name
    # backward: the producing kernel takes upsilon = c_d^(1/d) per output channel
    g = cases["conv->poly"]
    out, log = cc.redistribute(g, "backward")
    assert ("backward", "p", "k") in log
    u = np.sqrt(g["nodes"][1]["c"][..., 2])
    _close(out["nodes"][0]["W"], g["nodes"][0]["W"] * u[:, :, None, None, None])
    _close(out["nodes"][0]["b"], g["nodes"][0]["b"] * u)
    # forward: the consuming kernel takes upsilon = c_d per input channel
    g = cases["poly->conv"]
    out, log = cc.redistribute(g, "forward")
    u = g["nodes"][0]["c"][..., 2]
    _close(out["nodes"][1]["W"], g["nodes"][1]["W"] * u[:, None, :, None, None])
    _close(out["nodes"][0]["c"], g["nodes"][0]["c"] / u[..., None])


def test_average_pooling_donor():
    """Average pooling becomes a sum; the divisor moves into the consumer."""
    r = np.random.default_rng(3)
    M, C = 1, 2
    g = dict(members=M, image=(C, 4, 4), nodes=[
        dict(op="avgpool", name="pool", inp=["x"], out="p", div=4),
        dict(_conv(r, M, C), inp=["p"], out="o")])
    img = _rand(r, C, 4, 4)
    out, _ = cc.redistribute(g)
    assert out["nodes"][0]["div"] == 1
    _close(out["nodes"][1]["W"], g["nodes"][1]["W"] / 4)
    _close(og.forward(out, img), og.forward(g, img))


@pytest.mark.parametrize("order", ["conv_first", "poly_first"])
@pytest.mark.parametrize("direction", ["forward", "backward"])
@pytest.mark.parametrize("net", ["resnet", "vgg"])
def test_compiled_network_equals_trained_graph(order, direction, net):
    """Whole pipeline with exact clustering (every weight row its own
    centroid): the evaluator's description computes the trained network."""
    g = bn_resnet_graph(3, members=2) if net == "resnet" else bn_vgg_graph(4, members=2, pool_after=(0, 1))
    spec, log = cc.compile_network(g, k=4096, order=order, direction=direction)
    cases = {e[0] for e in log}
    if order == "conv_first":
        assert "case2" in cases
    elif net == "resnet":
        assert {"case1", "case3", "case4"} <= cases
    else:
        assert "case1" in cases
    ops = [L["op"] for L in spec["layers"]]
    assert "bn" not in ops and ops[-1] == "dense"
    for L in spec["layers"]:
        if L["op"] == "act":
            assert L["a_absorb"] == 1.0
    for s in range(2):
        img = gen.images(40 + s, 1, 3, 16, 16)[0]
        _close(spec_forward(spec, img), og.forward(g, img), 1e-10)


def test_clustered_network_approaches_the_trained_one():
    """Clustering is the one approximate step: the logits move, and move
    less as the codebook grows (random weights have no cluster structure, so
    the distance is larger than for a trained network)."""
    g = bn_resnet_graph(5, members=2)
    img = gen.images(50, 1, 3, 16, 16)[0]
    ref = og.forward(g, img)
    err = [np.max(np.abs(spec_forward(cc.compile_network(g, k=k)[0], img) - ref)) for k in (32, 128)]
    assert 1e-6 < err[1] < 0.5 * err[0]
    assert err[1] < 0.05 * np.max(np.abs(ref))


def test_slice_ensemble_clustering():
    r = np.random.default_rng(6)
    M = 3
    centres = np.array([[-1.0, 0.5, 2.0], [1.0, -1.0, 0.0], [0.0, 2.0, -2.0]])
    lab = r.integers(0, 3, 60)
    X = centres[lab] + r.normal(0, 0.01, (60, M))
    C, got = cc.lloyd(X, 3, seed=1)
    # well-separated blobs: the partition is the blobs', the centroids their means
    for c in range(3):
        sel = got == got[np.argmax(lab == c)]
        assert np.array_equal(sel, lab == c)
        _close(C[got[np.argmax(lab == c)]], X[lab == c].mean(axis=0))
    # codebook layout: W~[m, o, i, h, s] = codebook[s, idx[o, i, h, s], m], each row at its nearest centroid
    W = _rand(r, M, 4, 3, 3, 3)
    cb, idx = cc.cluster_slices(W, 8, seed=2)
    assert cb.shape == (3, 8, M) and idx.shape == (4, 3, 3, 3)
    for s in range(3):
        rows = W[..., s].reshape(M, -1).T
        d = ((rows[:, None, :] - cb[s][None]) ** 2).sum(axis=2)
        assert np.array_equal(idx[..., s].reshape(-1), d.argmin(axis=1))
    cb, idx = cc.cluster_slices(W, 64)  # 36 rows per slice <= 64: exact
    for s in range(3):
        _close(np.moveaxis(cb[s][idx[..., s]], -1, 0), W[..., s], 0.0)


def test_compile_errors():
    r = np.random.default_rng(7)
    M, C = 1, 2
    # a batch normalisation on the input (no convolution before, no activation after)
    g = dict(members=M, image=(C, 4, 4), nodes=[
        dict(op="bn", name="bn", inp=["x"], out="a", gamma=np.ones((M, C)), beta=np.zeros((M, C)),
             mean=np.zeros((M, C)), var=np.ones((M, C)), eps=1e-5),
        dict(_conv(r, M, C), inp=["a"], out="o")])
    with pytest.raises(cc.CompileError, match="batch normalisation"):
        cc.compile_network(g)
    # a bivariate activation that is not a polynomial of x + v y
    g = dict(members=M, image=(C, 4, 4), nodes=[
        dict(_conv(r, M, C), name="k1", inp=["x"], out="a"),
        dict(op="bipoly", name="s", inp=["a", "x"], out="s", c=_rand(r, M, C, 3, 3))])
    with pytest.raises(cc.CompileError, match="x \\+ v y"):
        cc.compile_network(g)
    # an activation as the output: per-channel leading coefficients cannot go
    # forward; backward they go into the convolution
    g = _chain(M, C, _conv(r, M, C), _poly(r, M, C))
    with pytest.raises(cc.CompileError, match="scale differs per channel"):
        cc.compile_network(g, direction="forward")
    spec, _ = cc.compile_network(g, k=4096, direction="backward")
    img = _rand(r, C, 4, 4)
    _close(spec_forward(spec, img)[0], og.forward(g, img)[0], 1e-11)
    with pytest.raises(cc.CompileError, match="unique"):
        cc.shapes(dict(members=1, image=(1, 4, 4), nodes=[dict(op="add", name="a", inp=["x", "x"], out="x")]))


def test_fixed_fitted_activation_becomes_per_channel():
    """A network trained with one quantisation-aware fitted activation
    (d = 2, b = 10, c = 2): Case 1 fusing gives every channel its own
    coefficients, and the compiled network still equals the trained one."""
    from paper_2509_22857_amd import qafit
    act = qafit.coefficients(2, 10, 2.0)
    g = bn_resnet_graph(8, members=2, act=act)
    assert all(np.array_equal(n["c"][0, 0], act) for n in g["nodes"] if n["op"] == "poly")
    spec, log = cc.compile_network(g, k=4096, order="poly_first")
    acts = [L for L in spec["layers"] if L["op"] == "act"]
    assert all(np.unique(L["b"]).size > 1 for L in acts)
    img = gen.images(70, 1, 3, 16, 16)[0]
    _close(spec_forward(spec, img), og.forward(g, img), 1e-10)


def test_batch_norm_after_dense_and_after_pooling():
    """Case 2 folds a BN that reads a dense layer; a BN after average pooling
    (not fusable) stays and receives the pooling's update as a polynomial of
    degree 1 -- until lowering, which refuses an unfused BN."""
    r = np.random.default_rng(9)
    M, C, K = 2, 3, 4

    def bn(name, inp, out, n):
        return dict(op="bn", name=name, inp=[inp], out=out, gamma=r.uniform(0.5, 1.5, (M, n)),
                    beta=_rand(r, M, n), mean=_rand(r, M, n), var=r.uniform(0.5, 2.0, (M, n)), eps=1e-5)

    g = dict(members=M, image=(C, 4, 4), nodes=[
        dict(_conv(r, M, C), name="k", inp=["x"], out="a"),
        dict(op="avgpool", name="pool", inp=["a"], out="p", div=4),
        bn("bnp", "p", "pb", C),
        dict(op="gap", name="gap", inp=["pb"], out="v", div=4),
        dict(op="dense", name="fc", inp=["v"], out="d", W=_rand(r, M, K, C), b=_rand(r, M, K)),
        bn("bnd", "d", "y", K)])
    img = _rand(r, C, 4, 4)
    ref = og.forward(g, img)
    f, log = cc.fuse(g)
    assert ("case2", "bnd", "fc") in log and any(n["op"] == "bn" for n in f["nodes"])
    _close(og.forward(f, img), ref, 1e-12)
    for direction in ("forward", "backward"):
        out, _ = cc.redistribute(f, direction)
        assert all(n["div"] == 1 for n in out["nodes"] if n["op"] in ("avgpool", "gap"))
        _close(og.forward(out, img), ref, 1e-11)
    with pytest.raises(cc.CompileError, match="batch normalisation"):
        cc.compile_network(g)
