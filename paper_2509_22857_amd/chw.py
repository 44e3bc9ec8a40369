"""Networks in the CHW layout: every channel of an image in one ciphertext.

Section 5.1 (Data Layout) names this packing as the alternative to the HW
layout the paper keeps.  Channel c's H x W grid takes the slot block
[c B, (c + 1) B), B = H W, pixel (r, x) at slot c B + r W + x; the N/2
slots hold N / (2 B) blocks, block b carrying channel b mod C (a C-channel
tensor is periodic with period C B), so a rotation by j B moves channel
(c + j) mod C onto block c.

A 3x3 'same' convolution from C_in to C_out channels (powers of two) is
then the diagonal method (Halevi and Shoup) over channels: for each channel
distance j < C_in and tap (dh, dw) one rotation of the input by
j B + dh W + dw, and one plaintext that carries, on every block b, the
weight of output channel b mod C_out from input channel (b + j) mod C_in
for that tap wherever the tap's source pixel is on the grid (zero
elsewhere: the zero padding).  Over the C_in distances block b meets every
input channel once, so it receives output channel b mod C_out and the output
is again periodic.  The rotation by j B is taken out of each distance's sum
(baby-step giant-step): the 9 tap rotations of the input are one hoisted
rotation group (one ModUp), each distance j sums its 9 products with the
plaintexts rotated right by j B in one plaintext multiply-accumulate, and
that sum is rotated by j B; 8 + C_in - 1 rotations instead of 9 C_in - 1,
and as many Galois keys.  The bias joins before the rescale.  The plaintexts are encoded
at scale q_l Delta / s for an input at level l and scale s, so every layer
leaves scale Delta.

Activation (monic quadratic x^2 + b x + c, Section 2.3): the relinearised
square plus x times the plaintext of b (at scale s) plus the plaintext of c
(at scale s^2), then a rescale.  Pooling: log2(B) doubling rotations leave
the sum of block c at slot c B.  Dense: per class, the pooled ciphertext
times the plaintext of that class's weights (at slots c B), log2(C)
doubling rotations by multiples of B leave the logit at slot 0, bias, rescale.

Every step runs in the library's kernels through its C-ABI (hoisted
rotation groups, plaintext MACs, products with relinearisation, additions,
rescales); this module only builds the plaintext slot vectors and sequences
the calls.
"""
from __future__ import annotations

import numpy as np

from . import ckks

_TAPS = [(dh, dw) for dh in (-1, 0, 1) for dw in (-1, 0, 1)]  # tap t = 3 (dh + 1) + (dw + 1)


class ChwNetwork:
    """The network of workloads.nets.chw_spec (conv C -> C1, activation,
    conv C1 -> C2, sum pooling, dense) on one context."""

    def __init__(self, ctx: ckks.Context, spec: dict, delta: float):
        self.ctx, self.spec, self.delta = ctx, spec, float(delta)
        self.C, self.H, self.W = spec["image"]
        self.B = self.H * self.W
        self.slots = ctx.N // 2
        self.nblocks = self.slots // self.B
        widths = (self.C, spec["conv1_w"].shape[0], spec["conv2_w"].shape[0])
        if any(c & (c - 1) for c in widths) or self.B & (self.B - 1):
            raise ValueError("CHW layout: channel counts and H W must be powers of two")
        if max(widths) * self.B > self.slots:
            raise ValueError(f"CHW layout: {max(widths)} channels of {self.B} slots exceed N/2 = {self.slots}")
        self.widths = widths
        self.logB = self.B.bit_length() - 1
        # valid-source masks per tap, [9][H][W]
        r = np.arange(self.H)[:, None]
        x = np.arange(self.W)[None, :]
        self.masks = np.stack([((r + dh >= 0) & (r + dh < self.H) & (x + dw >= 0) & (x + dw < self.W))
                               .astype(np.float64) for dh, dw in _TAPS])
        # encoded plaintexts by (layer, index, level, scale): a layer's inputs
        # arrive at one level and scale every time, so each is encoded once
        self._pts = {}

    def _pt(self, key, level: int, scale: float, slots, stream=None) -> ckks.Plaintext:
        k = (key, level, scale)
        if k not in self._pts:
            self._pts[k] = self.ctx.encode(slots() if callable(slots) else slots, level, scale, stream=stream)
        return self._pts[k]

    # ------------------------------------------------------------------ keys
    def rotation_steps(self, c_in: int) -> list[int]:
        """A convolution's rotations over c_in input channels: the 9 taps
        (the centre is the identity), then the channel distances 1 .. c_in - 1
        (multiples of B)."""
        return [dh * self.W + dw for dh, dw in _TAPS] + [j * self.B for j in range(1, c_in)]

    @property
    def steps(self) -> list[int]:
        """Every rotation step a run needs keys for (the identity excluded)."""
        st = set(self.rotation_steps(self.widths[0])) | set(self.rotation_steps(self.widths[1]))
        st.update(1 << i for i in range(self.logB))
        st.update(self.B << i for i in range(self.widths[2].bit_length() - 1))
        st.discard(0)
        return sorted(st)

    # ---------------------------------------------------------------- client
    def encrypt_image(self, keys: ckks.KeyPair, img: np.ndarray, stream_id: int) -> ckks.Ciphertext:
        z = np.tile(np.asarray(img, dtype=np.float64).reshape(self.C * self.B), self.slots // (self.C * self.B))
        L = len(self.ctx.q) - 1
        return self.ctx.encrypt(keys, self.ctx.encode(z, L, self.delta), stream_id)

    def decrypt_grid(self, keys: ckks.KeyPair, ct: ckks.Ciphertext, channels: int) -> np.ndarray:
        z = self.ctx.decode(self.ctx.decrypt(keys, ct), channels * self.B)
        return z.reshape(channels, self.H, self.W)

    def decrypt_logits(self, keys: ckks.KeyPair, cts) -> np.ndarray:
        return np.array([self.ctx.decode(self.ctx.decrypt(keys, c), 1)[0] for c in cts])

    # ---------------------------------------------------------------- layers
    def _per_block(self, v) -> np.ndarray:
        v = np.asarray(v, dtype=np.float64)
        return np.repeat(v[np.arange(self.nblocks) % len(v)], self.B)

    def _diag_slots(self, w: np.ndarray, j: int, t: int) -> np.ndarray:
        """Slots of the plaintext for channel distance j and tap t."""
        dh, dw = _TAPS[t]
        blk = np.arange(self.nblocks)
        wb = w[blk % w.shape[0], (blk + j) % w.shape[1], dh + 1, dw + 1]  # weight per block
        return (wb[:, None, None] * self.masks[t][None]).reshape(-1)

    def conv(self, keys, x: ckks.Ciphertext, w: np.ndarray, b: np.ndarray, name: str = "conv",
             stream=None) -> ckks.Ciphertext:
        ctx = self.ctx
        lv = x.level
        pt_scale = float(ctx.q[lv]) * self.delta / x.scale
        taps = [dh * self.W + dw for dh, dw in _TAPS]
        baby = ckks.rotate_many(ctx, keys, [x], taps, stream=stream)
        acc = None
        for j in range(w.shape[1]):
            # the plaintexts of distance j rotated right by j B (slot i holds
            # slot i - j B), so that the sum's rotation by j B lines them up
            pts = [self._pt((name, j, t), lv, pt_scale, lambda j=j, t=t: np.roll(self._diag_slots(w, j, t), j * self.B),
                            stream) for t in range(9)]
            inner = ckks.mac_plain_many(ctx, baby, pts, stream=stream)[0]
            if j:
                inner = ctx.rotate(keys, inner, [j * self.B], stream=stream)[0]
            acc = inner if acc is None else ctx.add(acc, inner, stream=stream)
        acc = ctx.add_plain(acc, self._pt((name, "bias"), lv, acc.scale, lambda: self._per_block(b), stream),
                            stream=stream)
        return ctx.rescale(acc, stream=stream)

    def act(self, keys, x: ckks.Ciphertext, b: np.ndarray, c: np.ndarray, name: str = "act",
            stream=None) -> ckks.Ciphertext:
        ctx = self.ctx
        sq = ckks.mul_relin_many(ctx, keys, [x], [x], stream=stream)[0]
        lin = ctx.mul_plain(x, self._pt((name, "b"), x.level, x.scale, lambda: self._per_block(b), stream),
                            stream=stream)
        y = ctx.add(sq, lin, stream=stream)
        y = ctx.add_plain(y, self._pt((name, "c"), x.level, y.scale, lambda: self._per_block(c), stream),
                          stream=stream)
        return ctx.rescale(y, stream=stream)

    def pool(self, keys, x: ckks.Ciphertext, stream=None) -> ckks.Ciphertext:
        ctx = self.ctx
        for i in range(self.logB):
            x = ctx.add(x, ctx.rotate(keys, x, [1 << i], stream=stream)[0], stream=stream)
        return x

    def dense(self, keys, x: ckks.Ciphertext, w: np.ndarray, bias: np.ndarray, name: str = "fc",
              stream=None) -> list:
        ctx = self.ctx
        lv = x.level
        pt_scale = float(ctx.q[lv]) * self.delta / x.scale

        def at(pos, v):
            z = np.zeros(self.slots)
            z[pos] = v
            return z

        C = w.shape[1]
        outs = []
        for k in range(w.shape[0]):
            wk = self._pt((name, k), lv, pt_scale, lambda k=k: at(slice(0, C * self.B, self.B), w[k]), stream)
            y = ctx.mul_plain(x, wk, stream=stream)
            for i in range(C.bit_length() - 1):
                y = ctx.add(y, ctx.rotate(keys, y, [self.B << i], stream=stream)[0], stream=stream)
            bk = self._pt((name, "bias", k), lv, y.scale, lambda k=k: at(0, bias[k]), stream)
            y = ctx.add_plain(y, bk, stream=stream)
            outs.append(ctx.rescale(y, stream=stream))
        return outs

    def run(self, keys, x: ckks.Ciphertext, stream=None) -> dict:
        """Outputs of every stage: conv1, act, conv2, pool and logits (one
        ciphertext per class, the logit at slot 0)."""
        s = self.spec
        out = {"conv1": self.conv(keys, x, s["conv1_w"], s["conv1_b"], "conv1", stream)}
        out["act"] = self.act(keys, out["conv1"], s["act_b"], s["act_c"], "act", stream)
        out["conv2"] = self.conv(keys, out["act"], s["conv2_w"], s["conv2_b"], "conv2", stream)
        out["pool"] = self.pool(keys, out["conv2"], stream)
        out["logits"] = self.dense(keys, out["pool"], s["fc_w"], s["fc_b"], "fc", stream)
        return out
