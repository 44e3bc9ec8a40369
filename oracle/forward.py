"""FP64 plaintext forward of a network spec -- TEST INFRASTRUCTURE ONLY.

The accuracy reference: the same clustered, redistributed network evaluated
in float64 for every ensemble member, with the paper's operator semantics:
zero-padded 'same' convolutions with stride (BN already folded), residual
sums, monic quadratic activations scaled by a_absorb, 2x2 sum pooling
(average divisor folded into the next layer), and a dense layer over the
per-channel sum of the final grid (global average pooling folded into w)
or, with a weight per grid position, over the flattened final map.
Written without reference to the generator's calibration forward.
"""
from __future__ import annotations

import numpy as np


def _expand_conv(ly):
    """[M][O][I][k][k] weights from the codebook + indices."""
    cb, idx = ly["codebook"], ly["idx"]
    k = idx.shape[2]
    M = cb.shape[2]
    O, I = idx.shape[0], idx.shape[1]
    W = np.zeros((M, O, I, k, k))
    for dh in range(k):
        for dw in range(k):
            W[:, :, :, dh, dw] = np.transpose(cb[dw][idx[:, :, dh, dw]], (2, 0, 1))
    return W


def _conv(x, W, bias, stride):
    """x: [I][H][W] one member; W: [O][I][k][k]."""
    I, H, Wd = x.shape
    O, _, k, _ = W.shape
    half = k // 2
    Ho, Wo = H // stride, Wd // stride
    y = np.zeros((O, Ho, Wo))
    for r in range(Ho):
        for c in range(Wo):
            for dh in range(-half, half + 1):
                ri = stride * r + dh
                if ri < 0 or ri >= H:
                    continue
                for dw in range(-half, half + 1):
                    ci = stride * c + dw
                    if ci < 0 or ci >= Wd:
                        continue
                    y[:, r, c] += W[:, :, dh + half, dw + half] @ x[:, ri, ci]
    if bias is not None:
        y += bias[:, None, None]
    return y


def forward(spec: dict, img: np.ndarray, capture: dict | None = None) -> np.ndarray:
    """img: [C][H][W] -> logits [M][K] (or the last tensor [M][C][H][W] for
    networks without a dense layer)."""
    M = spec["members"]
    outs = []
    for m in range(M):
        t = {"x": np.array(img, dtype=np.float64)}
        for ly in spec["layers"]:
            x = t[ly["inp"]]
            op = ly["op"]
            if op == "conv":
                W = _expand_conv(ly)[m]
                bias = None if ly.get("bias") is None else ly["bias"][m]
                y = _conv(x, W, bias, ly["stride"])
                if ly.get("short") is not None:
                    sh = ly["short"]
                    Ws = _expand_conv(sh)[m]
                    y = y + _conv(t[sh["inp"]], Ws, None, sh["stride"])
            elif op == "act":
                a = float(ly.get("a_absorb", 1.0))
                b = ly["b"][m][:, None, None]
                c = ly["c"][m][:, None, None]
                y = a * (x * x + b * x + c)
            elif op == "pool":
                y = x[:, 0::2, 0::2] + x[:, 0::2, 1::2] + x[:, 1::2, 0::2] + x[:, 1::2, 1::2]
            elif op == "dense":
                if np.ndim(ly["w"]) == 5:  # a weight per grid position (the flattened map)
                    y = np.einsum("kchw,chw->k", ly["w"][m], x)
                else:
                    y = ly["w"][m] @ x.sum(axis=(1, 2))
                y = y + (0.0 if ly.get("bias") is None else ly["bias"][m])
            else:
                raise ValueError(op)
            t[ly["out"]] = y
            if capture is not None:
                capture.setdefault(ly["out"], []).append(y)
        outs.append(t[spec["layers"][-1]["out"]])
    return np.array(outs)


def forward_chw(spec: dict, img: np.ndarray, capture: dict | None = None) -> np.ndarray:
    """The CHW-layout network of workloads.nets.chw_spec in float64: 'same'
    3x3 convolution, monic quadratic activation per channel, convolution,
    global sum pooling, dense.  img: [C][H][W] -> logits [K]; with capture,
    the intermediate tensors by stage name."""
    x = np.asarray(img, dtype=np.float64)
    y1 = _conv(x, spec["conv1_w"], spec["conv1_b"], 1)
    a = y1 * y1 + spec["act_b"][:, None, None] * y1 + spec["act_c"][:, None, None]
    y2 = _conv(a, spec["conv2_w"], spec["conv2_b"], 1)
    pooled = y2.sum(axis=(1, 2))
    logits = spec["fc_w"] @ pooled + spec["fc_b"]
    if capture is not None:
        capture.update(conv1=y1, act=a, conv2=y2, pool=pooled, logits=logits)
    return logits
