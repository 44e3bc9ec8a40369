"""Synthetic polynomial-activation CNNs, generated from a seed.

No trained weights or datasets exist here, so every network is drawn at
random with the shapes of the paper's models and then put into the form the
encrypted evaluator consumes (Sections 4 and 5 of the paper):
  * batch normalisation already folded into the convolutions (node fusing,
    Case 2): each convolution carries a bias;
  * quadratic activations a x^2 + b x + c with per-(channel, member)
    coefficients, made monic by weight redistribution (Section 4.2): the
    leading coefficient a moves forward into every consumer of the
    activation (the next convolution, the shortcut, the dense layer);
  * slice ensemble clustering (Sections 5.2-5.3): for every layer and kernel
    column, the weight vectors over the M ensemble members are replaced by
    the nearest of k centroids found by Lloyd's k-means (l2).
Before redistribution and clustering each convolution is standardised per
(member, output channel) over the calibration images -- what a folded batch
normalisation does -- which keeps the random network's signal input-dependent
and bounded.

The spec is a plain dict of numpy arrays.  The calibration forward below is
this module's own and serves only to scale the random weights; the oracle
has an independent forward used for accuracy checks.
"""
from __future__ import annotations

import numpy as np

from .gen import rng, images


# ----------------------------------------------------------------- k-means
def kmeans_rows(X: np.ndarray, k: int, iters: int = 50, seed: int = 0):
    """Lloyd's algorithm on the rows of X (n x M): returns (centroids k x M, labels n)."""
    n = X.shape[0]
    k = min(k, n)
    order = np.argsort(X.mean(axis=1), kind="stable")
    init = order[np.linspace(0, n - 1, k).round().astype(int)]
    C = X[init].copy()
    x2 = (X * X).sum(axis=1)[:, None]

    def assign(C):
        if X.shape[1] == 1:
            # one dimension: the nearest centroid is found between the
            # midpoints of the sorted centroids
            order = np.argsort(C[:, 0], kind="stable")
            cs = C[order, 0]
            return order[np.searchsorted((cs[1:] + cs[:-1]) / 2.0, X[:, 0])]
        d = x2 - 2.0 * (X @ C.T) + (C * C).sum(axis=1)[None, :]
        return d.argmin(axis=1)

    labels = np.zeros(n, dtype=np.int64)
    for _ in range(iters):
        labels = assign(C)
        counts = np.bincount(labels, minlength=k)
        sums = np.stack([np.bincount(labels, weights=X[:, m], minlength=k) for m in range(X.shape[1])], axis=1)
        nz = counts > 0
        C[nz] = sums[nz] / counts[nz, None]
    labels = assign(C)
    return C, labels


def cluster_conv(W: np.ndarray, k: int, seed: int = 0):
    """W: [M][O][I][kh][kw] -> codebook [kw][k][M], idx [O][I][kh][kw] (slice ensemble clustering)."""
    M, O, I, kh, kw = W.shape
    codebook = np.zeros((kw, k, M))
    idx = np.zeros((O, I, kh, kw), dtype=np.uint16)
    for col in range(kw):
        X = W[:, :, :, :, col].reshape(M, -1).T  # rows = (o, i, h), columns = members
        C, lab = kmeans_rows(X, k, seed=seed + col)
        codebook[col, :C.shape[0]] = C
        idx[:, :, :, col] = lab.reshape(O, I, kh)
    return codebook, idx


def conv_weights(codebook: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Expand a clustered convolution back to [M][O][I][kh][kw]."""
    kw = idx.shape[3]
    cols = [codebook[col][idx[:, :, :, col]] for col in range(kw)]  # each [O][I][kh][M]
    W = np.stack(cols, axis=3)  # [O][I][kh][kw][M]
    return np.moveaxis(W, -1, 0)


# ----------------------------------------------------------------- calibration forward
def _conv_fwd(x, W, b, stride):
    """x: [M][B][I][H][W]; W: [M][O][I][k][k]; b: [M][O] or None (zero 'same' padding)."""
    M, Bn, I, H, Wd = x.shape
    O, k = W.shape[1], W.shape[3]
    p = k // 2
    xp = np.pad(x, ((0, 0), (0, 0), (0, 0), (p, p), (p, p)))
    Ho, Wo = H // stride, Wd // stride
    y = np.zeros((M, Bn, O, Ho, Wo))
    for dh in range(k):
        for dw in range(k):
            patch = xp[:, :, :, dh:dh + H:stride, dw:dw + Wd:stride][:, :, :, :Ho, :Wo]
            # [M][B][I][Ho][Wo] x [M][O][I] as one batched matrix product per member
            pm = np.ascontiguousarray(np.moveaxis(patch, 2, -1)).reshape(M, -1, I)
            y += np.moveaxis((pm @ np.swapaxes(W[:, :, :, dh, dw], 1, 2)).reshape(M, Bn, Ho, Wo, O), -1, 2)
    if b is not None:
        y += b[:, None, :, None, None]
    return y


def _rms(x):
    return float(np.sqrt(np.mean(x * x)))


def _avgpool2(x):
    """2x2 average pooling of [M][B][C][H][W]."""
    M, Bn, C, H, W = x.shape
    return x.reshape(M, Bn, C, H // 2, 2, W // 2, 2).mean(axis=(4, 6))


def _standardise(g, xin, Wc, stride, pre_std):
    """Scale a convolution per (member, output channel) so its output over the
    calibration images has zero mean and standard deviation pre_std, plus a
    small random shift (a folded batch normalisation)."""
    y = _conv_fwd(xin, Wc, None, stride)  # [M][B][O][H][W]
    Mm, Bn, O = y.shape[0], y.shape[1], y.shape[2]
    u = np.moveaxis(y, 2, 1).reshape(Mm, O, -1)
    shift = g.normal(0.0, 0.1 * pre_std, (Mm, O))
    mu, sd = u.mean(axis=2), u.std(axis=2) + 1e-12
    s = pre_std / sd
    return Wc * s[:, :, None, None, None], -mu * s + shift


# ----------------------------------------------------------------- network builders
def _act_coeffs(g, M, C, b_range=(-0.5, 0.5), c_range=(-0.5, 0.5)):
    a = g.uniform(0.05, 0.2, (M, C))
    b = g.uniform(*b_range, (M, C))
    c = g.uniform(*c_range, (M, C))
    return a, b, c


def resnet_spec(seed: int = 0, members: int = 4, widths=(16, 32, 64), blocks: int = 3, classes: int = 100,
                image=(3, 32, 32), k: int = 64, calib: int = 16, name: str | None = None,
                block_slots: int | None = None, pre_std: float = 0.5) -> dict:
    """ResNet-style ensemble: conv1, len(widths) stages x `blocks` basic blocks
    (stride 2 at each new stage, 1x1 stride-2 projection shortcuts), global
    average pooling folded into the dense layer.

    Activations are ReLU-like quadratics (a in [0.05, 0.2], b in [0.4, 0.6],
    c in [-0.1, 0.1]) on pre-activations standardised to `pre_std`: deep
    random quadratic networks with larger curvature are chaotic (tiny input
    changes escape the fitted range, Section 2.3), which would make the FP64
    reference itself ill-conditioned."""
    g = rng(seed)
    act_b, act_c = (0.4, 0.6), (-0.1, 0.1)
    M = members
    Cin, H, W = image
    x = np.broadcast_to(images(seed + 1000, calib, Cin, H, W)[None], (M, calib, Cin, H, W)).copy()
    layers = []
    raw = []  # (kind, dict) before redistribution

    def new_conv(O, I, ksz, fan_scale=0.05):
        return g.normal(0.0, fan_scale, (M, O, I, ksz, ksz))

    # ---- raw network with calibration, stored as a list of ops.  Each
    # convolution is standardised per (member, output channel) over the
    # calibration images, as a folded batch normalisation would do: zero mean,
    # unit variance, plus a small random shift (the BN offset).
    def calibrate_conv(xin, Wc, stride, extra=None):
        if extra is None:
            return _standardise(g, xin, Wc, stride, pre_std)
        y = _conv_fwd(xin, Wc, None, stride)  # [M][B][O][H][W]
        Mm, Bn, O = y.shape[0], y.shape[1], y.shape[2]
        u = np.moveaxis(y, 2, 1).reshape(Mm, O, -1)
        shift = g.normal(0.0, 0.1 * pre_std, (Mm, O))
        v = np.moveaxis(extra, 2, 1).reshape(Mm, O, -1)
        uc = u - u.mean(axis=2, keepdims=True)
        vc = v - v.mean(axis=2, keepdims=True)
        A, Bq, Cq = (uc * uc).mean(axis=2), 2 * (uc * vc).mean(axis=2), (vc * vc).mean(axis=2) - pre_std ** 2
        disc = np.maximum(Bq * Bq - 4 * A * Cq, 0.0)
        s = (-Bq + np.sqrt(disc)) / (2 * A + 1e-30)
        s = np.where(s > 0, s, 0.5 * pre_std / np.sqrt(A + 1e-30))
        mean_z = s * u.mean(axis=2) + v.mean(axis=2)
        return Wc * s[:, :, None, None, None], -mean_z + shift

    def act_raw(xin, a, b, c):
        return a[:, None, :, None, None] * xin ** 2 + b[:, None, :, None, None] * xin + c[:, None, :, None, None]

    tensors = {"x": x}
    # conv1
    C0 = widths[0]
    W1, b1 = calibrate_conv(x, new_conv(C0, Cin, 3), 1)
    y = _conv_fwd(x, W1, b1, 1)
    a, b, c = _act_coeffs(g, M, C0, act_b, act_c)
    raw.append(("conv", dict(name="conv1", inp="x", out="c1", W=W1, b=b1, stride=1)))
    raw.append(("act", dict(name="act1", inp="c1", out="a1", a=a, b=b, c=c)))
    cur = act_raw(y, a, b, c)
    cur_name, cur_ch = "a1", C0
    for si, width in enumerate(widths):
        for bi in range(blocks):
            stride = 2 if (si > 0 and bi == 0) else 1
            tag = f"s{si}b{bi}"
            Wa, ba = calibrate_conv(cur, new_conv(width, cur_ch, 3), stride)
            ya = _conv_fwd(cur, Wa, ba, stride)
            aa, bb_, cc_ = _act_coeffs(g, M, width, act_b, act_c)
            ha = act_raw(ya, aa, bb_, cc_)
            if stride == 1 and width == cur_ch:
                Ws = np.broadcast_to(np.eye(width)[None, :, :, None, None], (M, width, width, 1, 1)).copy()
            else:
                Ws, _ = calibrate_conv(cur, g.normal(0.0, 0.05, (M, width, cur_ch, 1, 1)), stride)
                Ws = 0.5 * Ws
            short = _conv_fwd(cur, Ws, None, stride)
            Wb, bbias = calibrate_conv(ha, new_conv(width, width, 3), 1, extra=short)
            z = _conv_fwd(ha, Wb, bbias, 1) + short
            a2, b2, c2 = _act_coeffs(g, M, width, act_b, act_c)
            raw.append(("conv", dict(name=f"{tag}a", inp=cur_name, out=f"{tag}ca", W=Wa, b=ba, stride=stride)))
            raw.append(("act", dict(name=f"{tag}acta", inp=f"{tag}ca", out=f"{tag}ha", a=aa, b=bb_, c=cc_)))
            raw.append(("conv", dict(name=f"{tag}b", inp=f"{tag}ha", out=f"{tag}z", W=Wb, b=bbias, stride=1,
                                     short=dict(inp=cur_name, W=Ws, stride=stride))))
            raw.append(("act", dict(name=f"{tag}actb", inp=f"{tag}z", out=f"{tag}y", a=a2, b=b2, c=c2)))
            cur = act_raw(z, a2, b2, c2)
            cur_name, cur_ch = f"{tag}y", width
    # dense after global average pooling (divisor folded into w)
    Hf, Wf = cur.shape[3], cur.shape[4]
    pooled = cur.sum(axis=(3, 4))  # [M][B][C]
    Wd = g.normal(0.0, 0.05, (M, classes, cur_ch)) / (Hf * Wf)
    bd = g.normal(0.0, 0.1, (M, classes))
    logits = np.einsum("mbc,mkc->mbk", pooled, Wd) + bd[:, None, :]  # [M][B][K]
    s = 1.0 / max(_rms(logits), 1e-12)  # logit RMS 1 over the calibration images
    Wd, bd = Wd * s, bd * s
    raw.append(("dense", dict(name="fc", inp=cur_name, out="logits", W=Wd, b=bd)))
    return _finalise(raw, name or f"resnet_{'-'.join(map(str, widths))}x{blocks}_M{M}_k{k}", M, classes, image,
                     k, seed, block_slots)


def vgg_spec(seed: int = 0, widths=(64, 64, 128, 128, 256), pool_after=(1, 3), classes: int = 10,
             image=(3, 32, 32), k: int = 16, calib: int = 8, members: int = 1, name: str | None = None,
             pre_std: float = 0.5, hoist=None, dense: str = "gap") -> dict:
    """VGG-style network: one 3x3 convolution (stride 1) and one quadratic
    activation per entry of `widths`, 2x2 average pooling after the layers
    listed in pool_after, then the dense layer: over the global average
    pooling (dense="gap", folded into its weights) or over the flattened
    final map (dense="flatten": a weight N(0, 0.05) per class, channel and
    position, unclustered).  Weights N(0, 0.05) standardised per output
    channel (folded batch normalisation); activation coefficients
    a ~ U[0.05, 0.2] and b, c ~ U[-0.5, 0.5]; slice clustering with k
    centroids per layer."""
    g = rng(seed)
    M = members
    Cin, H, W = image
    x = np.broadcast_to(images(seed + 1000, calib, Cin, H, W)[None], (M, calib, Cin, H, W)).copy()
    raw = []
    cur, cur_name, cin = x, "x", Cin
    for li, width in enumerate(widths):
        Wc, bc = _standardise(g, cur, g.normal(0.0, 0.05, (M, width, cin, 3, 3)), 1, pre_std)
        y = _conv_fwd(cur, Wc, bc, 1)
        a, b, c = _act_coeffs(g, M, width)
        raw.append(("conv", dict(name=f"conv{li}", inp=cur_name, out=f"c{li}", W=Wc, b=bc, stride=1)))
        raw.append(("act", dict(name=f"act{li}", inp=f"c{li}", out=f"a{li}", a=a, b=b, c=c)))
        cur = a[:, None, :, None, None] * y ** 2 + b[:, None, :, None, None] * y + c[:, None, :, None, None]
        cur_name, cin = f"a{li}", width
        if li in pool_after:
            raw.append(("pool", dict(name=f"pool{li}", inp=cur_name, out=f"p{li}")))
            cur, cur_name = _avgpool2(cur), f"p{li}"
    Hf, Wf = cur.shape[3], cur.shape[4]
    if dense == "flatten":
        Wd = g.normal(0.0, 0.05, (M, classes, cin, Hf, Wf))
        bd = g.normal(0.0, 0.1, (M, classes))
        logits = np.einsum("mbchw,mkchw->mbk", cur, Wd) + bd[:, None, :]
    else:
        pooled = cur.sum(axis=(3, 4))
        Wd = g.normal(0.0, 0.05, (M, classes, cin)) / (Hf * Wf)
        bd = g.normal(0.0, 0.1, (M, classes))
        logits = np.einsum("mbc,mkc->mbk", pooled, Wd) + bd[:, None, :]
    s = 1.0 / max(_rms(logits), 1e-12)
    raw.append(("dense", dict(name="fc", inp=cur_name, out="logits", W=Wd * s, b=bd * s)))
    spec = _finalise(raw, name or f"vgg_{'-'.join(map(str, widths))}_M{M}_k{k}", M, classes, image, k, seed, None)
    return set_hoisting(spec, hoist)


def single_conv_spec(seed: int, I: int, O: int, k: int, M: int, H: int = 8, W: int = 8, block: int = 64,
                     stride: int = 1, hoist: str = "double") -> dict:
    """A network of one 3x3 convolution (codebook per kernel column with k
    centroids in R^M, uniform in [-0.3, 0.3]; uniform centroid choices; a
    bias per member and output), for layer-level parity cases."""
    g = rng(seed)
    codebook = g.uniform(-0.3, 0.3, (3, k, M))
    idx = g.integers(0, k, (O, I, 3, 3)).astype(np.uint16)
    bias = g.uniform(-0.5, 0.5, (M, O))
    layer = dict(op="conv", name="conv", inp="x", out="c", out_ch=O, in_ch=I, ksize=3, stride=stride,
                 codebook=codebook, idx=idx, bias=bias, hoist=hoist)
    return dict(name=f"conv_{I}x{O}_k{k}", members=M, classes=0, image=(I, H, W),
                layout=dict(block=block, row_stride=W), layers=[layer], k=k)


def act_dense_spec(seed: int, C: int, M: int, classes: int, H: int = 8, W: int = 8, block: int = 64) -> dict:
    """A network of one monic quadratic activation (b, c per member and
    channel, uniform in [-0.5, 0.5]) and the dense layer after global sum
    pooling (weights normal(0, 0.05) / (H W), bias normal(0, 0.1)), for
    layer-level parity cases of the activation, the slot-sum rotations and
    the dense contraction."""
    g = rng(seed)
    b = g.uniform(-0.5, 0.5, (M, C))
    c = g.uniform(-0.5, 0.5, (M, C))
    w = g.normal(0.0, 0.05, (M, classes, C)) / (H * W)
    bias = g.normal(0.0, 0.1, (M, classes))
    layers = [dict(op="act", name="act", inp="x", out="y", b=b, c=c, a_absorb=1.0),
              dict(op="dense", name="fc", inp="y", out="logits", w=w, bias=bias)]
    return dict(name=f"act_dense_{C}_K{classes}", members=M, classes=classes, image=(C, H, W),
                layout=dict(block=block, row_stride=W), layers=layers, k=0)


def chw_spec(seed: int, C: int = 8, H: int = 16, W: int = 16, classes: int = 4, C1: int | None = None,
             C2: int | None = None) -> dict:
    """A small network for the CHW layout (every channel of an image in one
    ciphertext): 3x3 'same' convolution C -> C1 (weights normal(0, 1 / (3
    sqrt(in channels))), bias uniform in [-0.2, 0.2]), monic quadratic
    activation (b, c uniform in [-0.5, 0.5] per channel), a second
    convolution C1 -> C2, global sum pooling and the dense layer (weights
    normal(0, 0.05) / (H W), bias normal(0, 0.1)).  Input images have C
    channels of H x W pixels; C1 and C2 default to C."""
    g = rng(seed)
    C1 = C if C1 is None else C1
    C2 = C1 if C2 is None else C2
    return dict(name=f"chw_{C}-{C1}-{C2}x{H}x{W}_K{classes}", layout="chw", image=(C, H, W), classes=classes,
                conv1_w=g.normal(0.0, 1.0 / (3.0 * np.sqrt(C)), (C1, C, 3, 3)), conv1_b=g.uniform(-0.2, 0.2, C1),
                act_b=g.uniform(-0.5, 0.5, C1), act_c=g.uniform(-0.5, 0.5, C1),
                conv2_w=g.normal(0.0, 1.0 / (3.0 * np.sqrt(C1)), (C2, C1, 3, 3)), conv2_b=g.uniform(-0.2, 0.2, C2),
                fc_w=g.normal(0.0, 0.05, (classes, C2)) / (H * W), fc_b=g.normal(0.0, 0.1, classes))


def set_hoisting(spec: dict, hoist) -> dict:
    """Mark the key-switching form of every 3x3 convolution: hoist is None
    (the default, double hoisting), "single"/"double" for all, or one entry
    per convolution in order.  The mark is part of the network description,
    read by both evaluators."""
    if hoist is None:
        return spec
    convs = [ly for ly in spec["layers"] if ly["op"] == "conv"]
    modes = [hoist] * len(convs) if isinstance(hoist, str) else list(hoist)
    if len(modes) != len(convs) or any(m not in ("single", "double") for m in modes):
        raise ValueError("hoist: 'single', 'double', or one of them per convolution")
    for ly, m in zip(convs, modes):
        ly["hoist"] = m
    return spec


def _finalise(raw, name, M, classes, image, k, seed, block_slots):
    """Weight redistribution (monic activations, a pushed forward) + clustering."""
    # consumers of each tensor: convs (main or shortcut) and dense
    act_scale = {}  # tensor name -> a [M][C] to multiply into consumers' input-channel weights
    for kind, d in raw:
        if kind == "act":
            act_scale[d["out"]] = d["a"]
        elif kind == "pool":
            # sum pooling: the average's divisor 1/4 moves into the consumers too
            act_scale[d["out"]] = 0.25 * act_scale[d["inp"]]
    layers = []
    for li, (kind, d) in enumerate(raw):
        if kind == "conv":
            W = d["W"].copy()
            if d["inp"] in act_scale:
                W = W * act_scale[d["inp"]][:, None, :, None, None]
            cb, ix = cluster_conv(W, k, seed=seed * 131 + li)
            L = dict(op="conv", name=d["name"], inp=d["inp"], out=d["out"], out_ch=W.shape[1], in_ch=W.shape[2],
                     ksize=W.shape[3], stride=d["stride"], codebook=cb, idx=ix, bias=d["b"].copy())
            if "short" in d:
                sh = d["short"]
                Ws = sh["W"].copy()
                if sh["inp"] in act_scale:
                    Ws = Ws * act_scale[sh["inp"]][:, None, :, None, None]
                scb, six = cluster_conv(Ws, k, seed=seed * 131 + li + 7)
                L["short"] = dict(inp=sh["inp"], ksize=1, stride=sh["stride"], out_ch=Ws.shape[1], in_ch=Ws.shape[2],
                                  codebook=scb, idx=six)
            layers.append(L)
        elif kind == "act":
            a = d["a"]
            layers.append(dict(op="act", name=d["name"], inp=d["inp"], out=d["out"], b=d["b"] / a, c=d["c"] / a,
                               a_absorb=1.0))
        elif kind == "dense":
            W = d["W"].copy()
            if d["inp"] in act_scale:
                sc = act_scale[d["inp"]][:, None, :]
                W = W * (sc[..., None, None] if W.ndim == 5 else sc)
            layers.append(dict(op="dense", name=d["name"], inp=d["inp"], out=d["out"], w=W, bias=d["b"].copy()))
        elif kind == "pool":
            layers.append(dict(op="pool", name=d["name"], inp=d["inp"], out=d["out"]))
    Cin, H, W = image
    B = block_slots or (1 << int(np.ceil(np.log2(H * W))))
    return dict(name=name, members=M, classes=classes, image=tuple(image), layout=dict(block=B, row_stride=W),
                layers=layers, k=k)


def tiny_spec(seed: int = 0) -> dict:
    """8x8x1 input, one 3x3 convolution with weights U[-1, 1], then the
    activation 0.125 x^2 + 0.5 x + 0.25 (leading coefficient absorbed into the
    scale; no next layer to receive it)."""
    g = rng(seed)
    w = g.uniform(-1.0, 1.0, (3, 3))
    codebook = np.zeros((3, 3, 1))
    idx = np.zeros((1, 1, 3, 3), dtype=np.uint16)
    for col in range(3):
        for h in range(3):
            codebook[col, h, 0] = w[h, col]
            idx[0, 0, h, col] = h
    a = 0.125
    layers = [
        dict(op="conv", name="conv", inp="x", out="c", out_ch=1, in_ch=1, ksize=3, stride=1, codebook=codebook,
             idx=idx, bias=None),
        dict(op="act", name="act", inp="c", out="y", b=np.array([[0.5 / a]]), c=np.array([[0.25 / a]]), a_absorb=a),
    ]
    return dict(name="tiny_conv_act", members=1, classes=0, image=(1, 8, 8), layout=dict(block=64, row_stride=8),
                layers=layers, k=3)


def pack_spec(spec: dict, images: int) -> dict:
    """Slot packing of several images per ciphertext: the same network with
    members * images member blocks, block p * M + m running member m on image
    p.  Every per-member array (codebook centroids, biases, activation
    coefficients, dense weights) is repeated once per packed image, so the
    evaluator computes, block by block, exactly what it computes for one image
    per ciphertext; only the client's packing puts a different image into each
    group of M blocks."""
    M, P = spec["members"], int(images)
    assert P >= 1

    def tile0(a):
        return None if a is None else np.tile(np.asarray(a), (P,) + (1,) * (np.ndim(a) - 1))

    def conv(d):
        d = dict(d)
        d["codebook"] = np.tile(d["codebook"], (1, 1, P))
        if d.get("bias") is not None:
            d["bias"] = tile0(d["bias"])
        if d.get("short") is not None:
            d["short"] = conv(d["short"])
        return d

    layers = []
    for ly in spec["layers"]:
        if ly["op"] == "conv":
            layers.append(conv(ly))
        elif ly["op"] == "act":
            layers.append(dict(ly, b=tile0(ly["b"]), c=tile0(ly["c"])))
        elif ly["op"] == "dense":
            layers.append(dict(ly, w=tile0(ly["w"]), bias=tile0(ly["bias"])))
        else:
            layers.append(dict(ly))
    out = dict(spec, members=M * P, layers=layers)
    out["packed"] = dict(images=P, members=M)
    return out
