"""A network in the CHW layout, on the oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module; the product path never does.

Layout (Section 5.1, Data Layout, the alternative to the HW layout that
packs several channels into one ciphertext): every channel of an image in one
ciphertext, channel c's H x W grid in the slot block [c B, (c + 1) B) with
B = H W, pixel (r, x) at slot c B + r W + x.  When C B is less than N/2
the C blocks are repeated to fill the N/2 slots (every slot vector of a
C-channel tensor periodic with period C B), so a rotation by j B brings
channel (c + j) mod C onto block c.

Convolution (3x3, 'same', stride 1, C_in -> C_out channels, both powers of
two) is the diagonal form of a matrix-vector product over channels (Halevi
and Shoup's diagonal method): with s_t = dh W + dw the slot offset of tap
t = (dh + 1, dw + 1),

    y = sum_{d < C_in} sum_{t < 9} P_{d,t} * Rot(x, d B + s_t),

where Rot is the left rotation of the slots and P_{d,t} holds, on every
block o of the slot vector, the weight w[o mod C_out][(o + d) mod C_in][t]
at every pixel (r, x) whose source pixel (r + dh, x + dw) lies on the grid,
and zero elsewhere (the zero padding of 'same').  As d runs over C_in
values, (o + d) mod C_in runs over every input channel, so block o receives
output channel o mod C_out: the output is periodic with period C_out B.  It
is evaluated in baby-step giant-step order (the rotation by d B taken out of
the inner sum; Q_{d,t} is P_{d,t} rotated right by d B, so that
Rot(Q * Rot(x, s_t), d B) = P * Rot(x, d B + s_t)):

    y = sum_{d < C_in} Rot(sum_{t < 9} Q_{d,t} * Rot(x, s_t), d B),

8 rotations of x (one per tap off the centre) and C_in - 1 rotations of the
inner sums, instead of 9 C_in - 1.  The bias (b[o mod C_out] on block o) is
added before the rescale.
Plaintexts are encoded at scale q_l Delta / s for an input at level l and
scale s, so every layer's output returns to scale Delta (up to the float
arithmetic of the scales).

The other layers: the monic quadratic activation x^2 + b x + c (Section 2.3)
as Relin(x (x) x) + x * P_b + P_c (b[c], c[c] on block c; P_b at the input's
scale s, P_c at s^2), then a rescale; global sum pooling as log2(B) doubling
rotations (slot c B then holds the sum of block c); the dense layer over C
channels, one ciphertext per class k: x * P_k with P_k = w[k][c] at slot
c B (c < C), log2(C)
doubling rotations by multiples of B (slot 0 then holds the logit), the bias
at slot 0, a rescale.
"""
from __future__ import annotations

import numpy as np

from .ckks import Ct, Oracle, SecretKey


def _taps():
    """(dh, dw) of the 9 taps, tap t = 3 (dh + 1) + (dw + 1)."""
    return [(t // 3 - 1, t % 3 - 1) for t in range(9)]


class OracleChw:
    def __init__(self, o: Oracle, spec: dict, delta: float):
        self.o, self.spec, self.delta = o, spec, float(delta)
        self.C, self.H, self.W = spec["image"]
        self.B = self.H * self.W
        self.n = o.N // 2
        self.nblk = self.n // self.B  # slot blocks
        self.widths = [self.C, spec["conv1_w"].shape[0], spec["conv2_w"].shape[0]]
        for c in self.widths + [self.B]:
            if c & (c - 1):
                raise ValueError("channel counts and H W must be powers of two (doubling rotations)")
        if max(self.widths) * self.B > self.n:
            raise ValueError("channels x H x W must not exceed N/2")

    # --------------------------------------------------------------- steps
    def conv_steps(self, c_in: int) -> list[int]:
        """The baby steps (taps) and giant steps (channel distances)."""
        return [dh * self.W + dw for (dh, dw) in _taps()] + [d * self.B for d in range(1, c_in)]

    def steps(self) -> list[int]:
        pool = [1 << j for j in range(self.B.bit_length() - 1)]
        chan = [self.B << j for j in range(self.widths[2].bit_length() - 1)]
        return sorted(set(self.conv_steps(self.widths[0])) | set(self.conv_steps(self.widths[1])) | set(pool)
                      | set(chan))

    # -------------------------------------------------------------- client
    def slots_of(self, img: np.ndarray) -> np.ndarray:
        z = np.zeros(self.n)
        for blk in range(self.nblk):
            z[blk * self.B:(blk + 1) * self.B] = np.asarray(img[blk % self.C], dtype=np.float64).reshape(-1)
        return z

    def encrypt_image(self, sk: SecretKey, img: np.ndarray, stream_id: int) -> Ct:
        pt = self.o.encode(self.slots_of(img), self.o.L, self.delta)
        return self.o.encrypt(pt, sk, stream_id)

    def grid_of(self, z: np.ndarray, channels: int) -> np.ndarray:
        """[channels][H][W] view of a decoded slot vector."""
        return np.asarray(z[:channels * self.B]).reshape(channels, self.H, self.W)

    # -------------------------------------------------------------- layers
    def _diagonal(self, w: np.ndarray, d: int, dh: int, dw: int) -> np.ndarray:
        c_out, c_in = w.shape[0], w.shape[1]
        z = np.zeros(self.n)
        for blk in range(self.nblk):
            oc, ic = blk % c_out, (blk + d) % c_in
            for r in range(self.H):
                if not 0 <= r + dh < self.H:
                    continue
                for x in range(self.W):
                    if 0 <= x + dw < self.W:
                        z[blk * self.B + r * self.W + x] = w[oc, ic, dh + 1, dw + 1]
        return z

    def _blocks(self, v: np.ndarray) -> np.ndarray:
        z = np.zeros(self.n)
        for blk in range(self.nblk):
            z[blk * self.B:(blk + 1) * self.B] = v[blk % len(v)]
        return z

    def conv(self, x: Ct, w: np.ndarray, b: np.ndarray, gk: dict) -> Ct:
        o = self.o
        pt_scale = float(o.q[x.level]) * self.delta / x.scale
        baby = [o.rotate(x, dh * self.W + dw, gk.get(o.galois_elt(dh * self.W + dw))) for (dh, dw) in _taps()]
        acc = None
        for d in range(w.shape[1]):
            inner = None
            for t, (dh, dw) in enumerate(_taps()):
                q = np.roll(self._diagonal(w, d, dh, dw), d * self.B)  # q[i] = P[i - d B]
                term = o.mul_plain(baby[t], o.encode(q, x.level, pt_scale))
                inner = term if inner is None else o.add(inner, term)
            if d:
                inner = o.rotate(inner, d * self.B, gk[o.galois_elt(d * self.B)])
            acc = inner if acc is None else o.add(acc, inner)
        acc = o.add_plain(acc, o.encode(self._blocks(b), x.level, acc.scale))
        return o.rescale(acc)

    def act(self, x: Ct, b: np.ndarray, c: np.ndarray, rlk: np.ndarray) -> Ct:
        o = self.o
        sq = o.relin(o.tensor(x, x), rlk)
        lin = o.mul_plain(x, o.encode(self._blocks(b), x.level, x.scale))
        y = o.add(sq, lin)
        y = o.add_plain(y, o.encode(self._blocks(c), x.level, y.scale))
        return o.rescale(y)

    def pool(self, x: Ct, gk: dict) -> Ct:
        o = self.o
        for j in range(self.B.bit_length() - 1):
            step = 1 << j
            x = o.add(x, o.rotate(x, step, gk[o.galois_elt(step)]))
        return x

    def dense(self, x: Ct, w: np.ndarray, bias: np.ndarray, gk: dict) -> list[Ct]:
        o = self.o
        pt_scale = float(o.q[x.level]) * self.delta / x.scale
        C = w.shape[1]
        outs = []
        for k in range(w.shape[0]):
            z = np.zeros(self.n)
            z[np.arange(C) * self.B] = w[k]
            y = o.mul_plain(x, o.encode(z, x.level, pt_scale))
            for j in range(C.bit_length() - 1):
                step = self.B << j
                y = o.add(y, o.rotate(y, step, gk[o.galois_elt(step)]))
            zb = np.zeros(self.n)
            zb[0] = bias[k]
            y = o.add_plain(y, o.encode(zb, y.level, y.scale))
            outs.append(o.rescale(y))
        return outs

    def run(self, x: Ct, rlk: np.ndarray, gk: dict) -> dict:
        """Every stage's output: conv1, act, conv2, pool (ciphertexts) and
        logits (one ciphertext per class, the logit at slot 0)."""
        s = self.spec
        out = {}
        out["conv1"] = self.conv(x, s["conv1_w"], s["conv1_b"], gk)
        out["act"] = self.act(out["conv1"], s["act_b"], s["act_c"], rlk)
        out["conv2"] = self.conv(out["act"], s["conv2_w"], s["conv2_b"], gk)
        out["pool"] = self.pool(out["conv2"], gk)
        out["logits"] = self.dense(out["pool"], s["fc_w"], s["fc_b"], gk)
        return out
