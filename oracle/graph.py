"""FP64 forward of a trained-network graph -- TEST INFRASTRUCTURE ONLY.

Evaluates the graph form the post-training compiler reads (batch
normalisations, polynomial activations of any degree, bivariate
activations, sums, average and global pooling, convolutions, dense layers,
diagonal scales) exactly as the operations are defined in Sections 4.1-4.2
of the paper, one ensemble member at a time, with plain loops.  It is the
reference the compiled network is checked against (the compiler's passes
must leave the network's function unchanged).  Written independently of the
compiler: it shares no code with it.
"""
from __future__ import annotations

import numpy as np


def _conv(x, W, b, stride):
    """Zero-padded 'same' convolution of x [I][H][W] by W [O][I][k][k]."""
    I, H, Wd = x.shape
    O, _, k, _ = W.shape
    half = k // 2
    y = np.zeros((O, H // stride, Wd // stride))
    for r in range(H // stride):
        for c in range(Wd // stride):
            for dh in range(k):
                for dw in range(k):
                    ri, ci = stride * r + dh - half, stride * c + dw - half
                    if 0 <= ri < H and 0 <= ci < Wd:
                        y[:, r, c] += W[:, :, dh, dw] @ x[:, ri, ci]
    if b is not None:
        y += b[:, None, None]
    return y


def _per_channel(v, x):
    """Broadcast a per-channel vector over x's grid (x [C] or [C][H][W])."""
    v = np.asarray(v, dtype=np.float64)
    return v.reshape(v.shape + (1,) * (x.ndim - 1))


def run(graph: dict, img: np.ndarray, member: int) -> np.ndarray:
    """Output of member `member` of the graph on one image [C][H][W]."""
    m = member
    t = {"x": np.array(img, dtype=np.float64)}
    for n in graph["nodes"]:
        x = t[n["inp"][0]]
        op = n["op"]
        if op == "conv":
            y = _conv(x, n["W"][m], None if n.get("b") is None else n["b"][m], n["stride"])
        elif op == "dense":
            y = n["W"][m] @ x + (0.0 if n.get("b") is None else n["b"][m])
        elif op == "scale":
            y = _per_channel(n["s"][m], x) * x
        elif op == "bn":
            # (x - mean) / sqrt(var + eps) * gamma + beta, per channel
            y = ((x - _per_channel(n["mean"][m], x)) / np.sqrt(_per_channel(n["var"][m], x) + n["eps"])
                 * _per_channel(n["gamma"][m], x) + _per_channel(n["beta"][m], x))
        elif op == "poly":
            c = n["c"][m]
            y = np.zeros_like(x)
            for i in range(c.shape[-1]):  # sum_i c_i x^i, powers by repeated products
                p = np.ones_like(x)
                for _ in range(i):
                    p = p * x
                y = y + _per_channel(c[:, i], x) * p
        elif op == "bipoly":
            yv = t[n["inp"][1]]
            c = n["c"][m]
            y = np.zeros_like(x)
            for i in range(3):
                for j in range(3 - i):
                    y = y + _per_channel(c[:, i, j], x) * x ** i * yv ** j
        elif op == "add":
            y = x + t[n["inp"][1]]
        elif op == "avgpool":
            C, H, W = x.shape
            y = np.zeros((C, H // 2, W // 2))
            for r in range(H // 2):
                for c in range(W // 2):
                    y[:, r, c] = x[:, 2 * r:2 * r + 2, 2 * c:2 * c + 2].sum(axis=(1, 2)) / n["div"]
        elif op == "gap":
            y = x.sum(axis=(1, 2)) / n["div"]
        else:
            raise ValueError(op)
        if "absorb" in n:
            a = np.asarray(n["absorb"], dtype=np.float64)
            y = y * (_per_channel(a[m], y) if a.ndim == 2 else a)
        t[n["out"]] = y
    return t[graph["nodes"][-1]["out"]]


def forward(graph: dict, img: np.ndarray) -> np.ndarray:
    """Outputs of every member: [M][...]."""
    return np.array([run(graph, img, m) for m in range(graph["members"])])
