"""Seeded synthetic trained-network graphs for the post-training compiler.

No trained weights exist here, so a "trained" network is drawn at random in
the graph form the compiler reads: convolutions followed by batch
normalisations whose statistics (mean, variance) are those of the batch of
calibration images -- what a trained network's running statistics hold --
with learnable gamma, beta drawn at random; ReLU-like quadratic activations
c2 x^2 + c1 x + c0 (c2 in [0.05, 0.2], c1 in [0.4, 0.6], c0 in [-0.1, 0.1]);
residual sums of two batch-normalised branches (projection shortcut) or of
a batch-normalised branch and the block input (identity shortcut); average
pooling; global average pooling and a dense layer.  Every parameter has a
leading axis over the M ensemble members.

The calibration forward below is this module's own and only sets the batch
statistics; the oracle's graph forward is separate.
"""
from __future__ import annotations

import numpy as np

from .gen import images, rng
from .nets import _conv_fwd


def _bcast(v, x):
    """[M][C] -> broadcastable over x [M][B][C][...]."""
    return v.reshape(v.shape[:1] + (1,) + v.shape[1:2] + (1,) * (x.ndim - 3))


def _calib(n, t):
    """One node on the calibration batch (tensors [M][B][C][H][W] or [M][B][C])."""
    x = t[n["inp"][0]]
    op = n["op"]
    if op == "conv":
        return _conv_fwd(x, n["W"], n.get("b"), n["stride"])
    if op == "bn":
        b1 = n["gamma"] / np.sqrt(n["var"] + n["eps"])
        return _bcast(b1, x) * (x - _bcast(n["mean"], x)) + _bcast(n["beta"], x)
    if op == "poly":
        c = n["c"]
        return sum(_bcast(c[..., i], x) * x ** i for i in range(c.shape[-1]))
    if op == "add":
        return x + t[n["inp"][1]]
    if op == "avgpool":
        M, B, C, H, W = x.shape
        return x.reshape(M, B, C, H // 2, 2, W // 2, 2).sum(axis=(4, 6)) / n["div"]
    if op == "gap":
        return x.sum(axis=(3, 4)) / n["div"]
    if op == "dense":
        y = np.einsum("mbc,mkc->mbk", x, n["W"])
        return y if n.get("b") is None else y + n["b"][:, None, :]
    raise ValueError(op)


class _Builder:
    def __init__(self, seed, members, image, calib, pre_std, act=None):
        self.act_poly = None if act is None else np.asarray(act, dtype=np.float64)
        self.g = rng(seed)
        self.M = members
        self.pre_std = pre_std
        C, H, W = image
        x = images(seed + 2000, calib, C, H, W)
        self.t = {"x": np.broadcast_to(x[None], (members,) + x.shape).copy()}
        self.nodes = []

    def add(self, n):
        self.nodes.append(n)
        self.t[n["out"]] = _calib(n, self.t)
        return n["out"]

    def conv(self, name, inp, O, k, stride=1, bias=True):
        I = self.t[inp].shape[2]
        W = self.g.normal(0.0, 0.3 / np.sqrt(I * k * k), (self.M, O, I, k, k))
        b = self.g.normal(0.0, 0.05, (self.M, O)) if bias else None
        return self.add(dict(op="conv", name=name, inp=[inp], out=name, W=W, b=b, stride=stride))

    def bn(self, name, inp):
        x = self.t[inp]
        mean = np.moveaxis(x, 2, 1).reshape(self.M, x.shape[2], -1).mean(axis=2)
        var = np.moveaxis(x, 2, 1).reshape(self.M, x.shape[2], -1).var(axis=2)
        C = x.shape[2]
        gamma = self.pre_std * self.g.uniform(0.8, 1.2, (self.M, C))
        beta = self.g.normal(0.0, 0.1 * self.pre_std, (self.M, C))
        return self.add(dict(op="bn", name=name, inp=[inp], out=name, gamma=gamma, beta=beta, mean=mean, var=var,
                             eps=1e-5))

    def act(self, name, inp, degree=2):
        C = self.t[inp].shape[2]
        if self.act_poly is not None:  # one fixed activation polynomial everywhere
            c = np.broadcast_to(self.act_poly, (self.M, C, len(self.act_poly))).copy()
            return self.add(dict(op="poly", name=name, inp=[inp], out=name, c=c))
        c = np.zeros((self.M, C, degree + 1))
        c[..., 0] = self.g.uniform(-0.1, 0.1, (self.M, C))
        c[..., 1] = self.g.uniform(0.4, 0.6, (self.M, C))
        c[..., 2] = self.g.uniform(0.05, 0.2, (self.M, C))
        if degree > 2:
            c[..., 3:] = self.g.uniform(0.01, 0.03, (self.M, C, degree - 2))
        return self.add(dict(op="poly", name=name, inp=[inp], out=name, c=c))

    def head(self, inp, classes):
        x = self.t[inp]
        H, W = x.shape[3], x.shape[4]
        p = self.add(dict(op="gap", name="gap", inp=[inp], out="gap", div=H * W))
        C = self.t[p].shape[2]
        W_ = self.g.normal(0.0, 1.0 / np.sqrt(C), (self.M, classes, C))
        b = self.g.normal(0.0, 0.1, (self.M, classes))
        y = np.einsum("mbc,mkc->mbk", self.t[p], W_) + b[:, None, :]
        s = 1.0 / max(float(np.sqrt(np.mean(y * y))), 1e-12)  # logit RMS 1 on the calibration images
        return self.add(dict(op="dense", name="fc", inp=[p], out="logits", W=W_ * s, b=b * s))


def bn_resnet_graph(seed: int = 0, members: int = 2, widths=(4, 8), blocks: int = 1, classes: int = 10,
                    image=(3, 16, 16), calib: int = 4, pre_std: float = 0.5, act=None) -> dict:
    """ResNet-style: conv-BN-act, then per stage `blocks` basic blocks
    (conv-BN-act-conv-BN, plus the shortcut -- identity, or a 1x1 stride-2
    projection conv-BN at a new stage -- then the activation of the sum),
    global average pooling and a dense layer.  act = (c0, c1, c2, ...) puts
    that one polynomial at every activation (a network trained with a fixed
    fitted activation); otherwise coefficients are drawn per channel."""
    b = _Builder(seed, members, image, calib, pre_std, act)
    cur = b.act("act1", b.bn("bn1", b.conv("conv1", "x", widths[0], 3, bias=False)))
    ch = widths[0]
    for si, w in enumerate(widths):
        for bi in range(blocks):
            tag = f"s{si}b{bi}"
            stride = 2 if (si > 0 and bi == 0) else 1
            h = b.act(f"{tag}acta", b.bn(f"{tag}bna", b.conv(f"{tag}ca", cur, w, 3, stride)))
            z = b.bn(f"{tag}bnb", b.conv(f"{tag}cb", h, w, 3))
            if stride == 1 and w == ch:
                short = cur
            else:
                short = b.bn(f"{tag}bns", b.conv(f"{tag}cs", cur, w, 1, stride, bias=False))
            s = b.add(dict(op="add", name=f"{tag}add", inp=[z, short], out=f"{tag}add"))
            cur, ch = b.act(f"{tag}actb", s), w
    b.head(cur, classes)
    return dict(members=members, image=tuple(image), nodes=b.nodes)


def bn_vgg_graph(seed: int = 0, members: int = 1, widths=(4, 8, 8), pool_after=(0,), classes: int = 10,
                 image=(3, 16, 16), calib: int = 4, pre_std: float = 0.5, degree: int = 2) -> dict:
    """VGG-style: conv-BN-act per entry of `widths`, 2x2 average pooling after
    the layers in pool_after, global average pooling and a dense layer.
    degree > 2 gives activations the evaluator does not run (for checks of
    fusing and redistribution alone)."""
    b = _Builder(seed, members, image, calib, pre_std)
    cur = "x"
    for li, w in enumerate(widths):
        cur = b.act(f"act{li}", b.bn(f"bn{li}", b.conv(f"conv{li}", cur, w, 3)), degree=degree)
        if li in pool_after:
            cur = b.add(dict(op="avgpool", name=f"pool{li}", inp=[cur], out=f"pool{li}", div=4))
    b.head(cur, classes)
    return dict(members=members, image=tuple(image), nodes=b.nodes)
