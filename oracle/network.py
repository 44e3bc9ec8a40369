"""Oracle evaluation of an encrypted CNN -- TEST INFRASTRUCTURE ONLY.

Written independently of the GPU runner from the paper's method:
  * HW layout (Section 5.1): channel -> ciphertext, member m's copy of the
    grid in slot block m, pixel (r, c) at slot m*block + gap*(r*row_stride + c);
  * convolution: every weight w[o][i][dh][dw] (a vector over members, taken
    from the clustered codebook, Sections 5.2-5.3) is encoded on the output
    slots whose input pixel lies inside the image, and multiplies the input
    rotated by gap*(dh*row_stride + dw); all products are summed, plus the
    bias on the output grid.  This is the unclustered sum; grouping equal
    centroids first gives the same ring element.  A 3x3 layer's rotated
    inputs stay in Q_l u P and are summed there with one ModDown per output
    (double hoisting), or, for a layer marked single-hoisted, each is a
    complete rotation back in Q_l before the sum;
  * activation x^2 + b x + c: t = x + b, y = Relin(x * t) + c (Section 4.2
    makes it monic), scale s^2 / a_absorb;
  * dense: rotation sums over the grid, then per class the weighted sum of
    the channel sums, plus bias (member values at slot m*block); with a
    weight per grid position (the flattened map), per class the weighted
    products of the channels plus the bias first, then the rotation sums;
  * tower reuse (Section 4.3): rescale after a multiplicative layer iff the
    sublevel of its scale exceeds the sublevel of the prime to drop;
  * slice-shared layout (layout flag "slice_shared"; Section 5.2: the
    weights of one kernel column across the layer's filters share an
    encoding): every member block keeps zero rows below its image, so a
    vertical tap that leaves the image reads zeros and needs no mask; the
    plaintext of a weight then depends only on its kernel column (the
    horizontal mask), and the three taps of a column share it.  Keeping the
    spare rows zero asks every layer to leave them zero: the activation's
    constant term is placed on the image's grid only.
"""
from __future__ import annotations

import math

import numpy as np

from .ckks import Oracle, Ct, Pt, SecretKey


def _lam(s, delta):
    return int(round(math.log2(s) / math.log2(delta)))


class OracleNetwork:
    def __init__(self, orc: Oracle, spec: dict, delta: float, target: float, in_scale: float):
        self.o, self.spec = orc, spec
        self.delta, self.target, self.in_scale = delta, target, in_scale
        C, H, W = spec["image"]
        self.B = spec["layout"]["block"]
        self.W0 = spec["layout"]["row_stride"]
        self.M = spec["members"]
        self.input_grid = dict(gap=1, H=H, W=W)
        self.slice_shared = bool(spec["layout"].get("slice_shared", False))

    def _check_spare_rows(self, grid):
        """Slice-shared layout: the row after the image's last row and the
        row before its first (the previous block's last rows) must hold only
        zeros at the grid's gap, i.e. a block has at least gap*(H + 1) rows."""
        rows = self.B // self.W0
        if rows < grid["gap"] * (grid["H"] + 1):
            raise ValueError(f"slice-shared layout needs {grid['gap'] * (grid['H'] + 1)} rows per block, "
                             f"the layout has {rows}")

    # ------------------------------------------------------------ slots
    def _slot(self, m, r, c, gap):
        return m * self.B + gap * (r * self.W0 + c)

    def _vec(self):
        return np.zeros(self.o.N // 2)

    def encode(self, v, level, scale) -> Pt:
        return self.o.encode(v, level, scale)

    # ------------------------------------------------------------ levels and scales (Section 4.3)
    def _rescale_needed(self, level, scale):
        """Tower reuse: rescale iff the sublevel of the scale exceeds the
        sublevel of the prime that would be dropped."""
        return level >= 1 and _lam(scale, self.delta) > _lam(float(self.o.q[level]), self.delta)

    def _pt_scale(self, level, s):
        """Plaintext scale of a convolution or dense layer whose input has
        scale s at `level`: the product's scale divided by q_level is the
        target scale."""
        return (self.target * float(self.o.q[level])) / s

    def _out_scale(self, ly, level, s):
        """Scale of a layer's output before the optional rescale."""
        op = ly["op"]
        if op in ("conv", "dense"):
            return s * self._pt_scale(level, s)
        if op == "act":
            return (s * s) / float(ly.get("a_absorb", 1.0))
        return s

    def schedule(self):
        """The level and scale of every tensor, from the rules run() applies,
        without ciphertexts: a list of dicts (name, op, level_in, scale_in,
        scale_out before rescaling, rescale, level_out, scale_out_final)."""
        state = {"x": (self.o.L, float(self.in_scale))}
        out = []
        for ly in self.spec["layers"]:
            level, s = state[ly["inp"]]
            S = self._out_scale(ly, level, s)
            resc = ly["op"] != "pool" and self._rescale_needed(level, S)
            lo, so = (level - 1, S / float(self.o.q[level])) if resc else (level, S)
            if lo < 0:
                raise ValueError("chain too short for this network")
            state[ly["out"]] = (lo, so)
            out.append(dict(name=ly["name"], op=ly["op"], level_in=level, scale_in=s, scale_out=S, rescale=resc,
                            level_out=lo, scale_out_final=so))
        return out

    # ------------------------------------------------------------ client
    def encrypt_image(self, sk: SecretKey, img: np.ndarray, stream_base: int):
        C, H, W = self.spec["image"]
        cts = []
        for c in range(C):
            v = self._vec()
            for m in range(self.M):
                for r in range(H):
                    for col in range(W):
                        v[self._slot(m, r, col, 1)] = img[c, r, col]
            pt = self.encode(v, self.o.L, self.in_scale)
            cts.append(self.o.encrypt(pt, sk, stream_base + c))
        return cts

    # ------------------------------------------------------------ layers
    def conv(self, xs, grid, ly, pt_scale, bias_scale, gkeys, with_bias=True):
        o = self.o
        k = ly["ksize"]
        half = k // 2
        s = ly["stride"]
        g, H, W = grid["gap"], grid["H"], grid["W"]
        Ho, Wo, go = H // s, W // s, g * s
        level = xs[0].level
        cb, idx = ly["codebook"], ly["idx"]

        # with the slice-shared layout a 3x3 weight's plaintext depends on its
        # column only: vertical taps past the image read the zero rows
        shared = self.slice_shared and k == 3
        if shared:
            self._check_spare_rows(grid)

        def mask(dh, dw, wvec):
            # a weight vector on the output slots whose input pixel is inside
            # (slice-shared: whose input column is inside)
            v = self._vec()
            for m in range(self.M):
                for r in range(Ho):
                    if not shared and not 0 <= s * r + dh < H:
                        continue
                    for c in range(Wo):
                        if 0 <= s * c + dw < W:
                            v[self._slot(m, r, c, go)] = wvec[m]
            return v

        taps = [(dh, dw) for dh in range(-half, half + 1) for dw in range(-half, half + 1)]
        outs = []
        if k == 1:
            # a single tap of step 0: plain products (no key switching)
            cache = {}
            for oc in range(ly["out_ch"]):
                acc = None
                for i, x in enumerate(xs):
                    wvec = cb[0][idx[oc, i, 0, 0]]
                    key = tuple(wvec)
                    if key not in cache:
                        cache[key] = self.encode(mask(0, 0, wvec), level, pt_scale)
                    term = o.mul_plain(x, cache[key])
                    acc = term if acc is None else o.add(acc, term)
                outs.append(acc)
        elif ly.get("hoist", "double") == "single":
            # single hoisting: every rotated input is a complete rotation
            # (key switch with its own ModDown, back in Q_l), the products
            # with plaintexts encoded over Q_l are summed there
            rot = {}
            for i, x in enumerate(xs):
                for dh, dw in taps:
                    step = g * (dh * self.W0 + dw)
                    gk = gkeys[o.galois_elt(step)] if step else None
                    rot[(i, dh, dw)] = o.rotate(x, step, gk)
            cache = {}
            for oc in range(ly["out_ch"]):
                acc = None
                for i in range(ly["in_ch"]):
                    for dh, dw in taps:
                        wvec = cb[dw + half][idx[oc, i, dh + half, dw + half]]
                        key = (0 if shared else dh, dw, tuple(wvec))
                        if key not in cache:
                            cache[key] = self.encode(mask(dh, dw, wvec), level, pt_scale)
                        term = o.mul_plain(rot[(i, dh, dw)], cache[key])
                        acc = term if acc is None else o.add(acc, term)
                outs.append(acc)
        else:
            # double hoisting: every rotated input stays in the extended basis
            # Q_l u P as P*sigma(c0) + u0 and u1 (the key switch without its
            # ModDown; the identity tap is P*x), the products with plaintexts
            # encoded over Q_l u P are summed there, and one ModDown per
            # output polynomial brings the sum back to Q_l.
            nl = level + 1
            nt = nl + o.np_
            prime = [l if l < nl else o.nq + (l - nl) for l in range(nt)]
            P_mod = []
            for l in range(nl):
                v = 1
                for pk in o.p:
                    v = (v * pk) % o.q[l]
                P_mod.append(v)

            def times_P(a, l):
                return ((a.astype(object) * P_mod[l]) % o.q[l]).astype(np.uint64)

            ext = {}
            for i, x in enumerate(xs):
                for dh, dw in taps:
                    step = g * (dh * self.W0 + dw)
                    R = np.zeros((2, nt, o.N), dtype=np.uint64)
                    if step == 0:
                        for p in range(2):
                            for l in range(nl):
                                R[p, l] = times_P(x.data[p, l], l)
                    else:
                        gel = o.galois_elt(step)
                        R = o.keyswitch_ext(x.data[1], level, gkeys[gel], gel)
                        for l in range(nl):
                            sa = times_P(o.automorphism(x.data[0, l], gel, l), l)
                            R[0, l] = o._add(R[0, l], sa, np.uint64(o.q[l]))
                    ext[(i, dh, dw)] = R
            cache = {}
            for oc in range(ly["out_ch"]):
                acc = np.zeros((2, nt, o.N), dtype=np.uint64)
                for i in range(ly["in_ch"]):
                    for dh, dw in taps:
                        wvec = cb[dw + half][idx[oc, i, dh + half, dw + half]]
                        key = (0 if shared else dh, dw, tuple(wvec))
                        if key not in cache:
                            cache[key] = o.encode_ext(mask(dh, dw, wvec), level, pt_scale)
                        pt = cache[key]
                        R = ext[(i, dh, dw)]
                        for p in range(2):
                            for l in range(nt):
                                prod = o.polymul(R[p, l], pt[l], prime[l])
                                acc[p, l] = o._add(acc[p, l], prod, np.uint64(o.mod[prime[l]]))
                y = np.stack([o.moddown(acc[p], level) for p in range(2)])
                outs.append(Ct(y, level, xs[0].scale * pt_scale))
        for oc in range(ly["out_ch"]):
            acc = outs[oc]
            if with_bias and ly.get("bias") is not None:
                v = self._vec()
                for m in range(self.M):
                    for r in range(Ho):
                        for c in range(Wo):
                            v[self._slot(m, r, c, go)] = ly["bias"][m, oc]
                acc = o.add_plain(acc, self.encode(v, level, bias_scale))
            outs[oc] = acc
        return outs, dict(gap=go, H=Ho, W=Wo)

    def act(self, xs, ly, rlk, grid=None):
        o = self.o
        out = []
        for ch, x in enumerate(xs):
            if self.slice_shared:
                # the spare rows stay zero: b multiplies x (zero there), and c
                # is placed on the grid's slots only
                if self.M == 1:
                    t = o.add_const(x, float(ly["b"][0, ch]))
                else:
                    v = self._vec()
                    for m in range(self.M):
                        v[m * self.B:(m + 1) * self.B] = ly["b"][m, ch]
                    t = o.add_plain(x, self.encode(v, x.level, x.scale))
                y = o.relin(o.tensor(x, t), rlk)
                v = self._vec()
                for m in range(self.M):
                    for r in range(grid["H"]):
                        for c in range(grid["W"]):
                            v[self._slot(m, r, c, grid["gap"])] = ly["c"][m, ch]
                y = o.add_plain(y, self.encode(v, y.level, y.scale))
                out.append(Ct(y.data, y.level, self._out_scale(ly, x.level, x.scale)))
                continue
            if self.M == 1:
                t = o.add_const(x, float(ly["b"][0, ch]))
            else:
                v = self._vec()
                for m in range(self.M):
                    v[m * self.B:(m + 1) * self.B] = ly["b"][m, ch]
                t = o.add_plain(x, self.encode(v, x.level, x.scale))
            y = o.relin(o.tensor(x, t), rlk)
            if self.M == 1:
                y = o.add_const(y, float(ly["c"][0, ch]))
            else:
                v = self._vec()
                for m in range(self.M):
                    v[m * self.B:(m + 1) * self.B] = ly["c"][m, ch]
                y = o.add_plain(y, self.encode(v, y.level, y.scale))
            y = Ct(y.data, y.level, self._out_scale(ly, x.level, x.scale))
            out.append(y)
        return out

    def dense(self, xs, grid, ly, pt_scale, bias_scale, gkeys):
        o = self.o
        g, H, W = grid["gap"], grid["H"], grid["W"]
        steps = [g * (1 << j) for j in range(int(math.log2(W)))] + \
                [g * self.W0 * (1 << j) for j in range(int(math.log2(H)))]
        if np.ndim(ly["w"]) == 5:
            return self._dense_spatial(xs, g, H, W, steps, ly, pt_scale, bias_scale, gkeys)
        sums = []
        for x in xs:
            S = x
            for st in steps:
                S = o.add(S, o.rotate(S, st, gkeys[o.galois_elt(st)]))
            sums.append(S)
        K = ly["w"].shape[1]
        level = xs[0].level
        outs = []
        for kk in range(K):
            acc = None
            for c, S in enumerate(sums):
                if self.M == 1:
                    # one member: a constant multiplier (only slot 0 is read)
                    term = o.mul_const(S, ly["w"][0, kk, c], pt_scale)
                else:
                    v = self._vec()
                    for m in range(self.M):
                        v[m * self.B] = ly["w"][m, kk, c]
                    term = o.mul_plain(S, self.encode(v, level, pt_scale))
                acc = term if acc is None else o.add(acc, term)
            if ly.get("bias") is not None:
                if self.M == 1:
                    r = o.const_residues(ly["bias"][0, kk], bias_scale, level + 1)
                    data = acc.data.copy()
                    for l in range(level + 1):
                        data[0, l, 0] = np.uint64((int(data[0, l, 0]) + int(r[l])) % o.q[l])
                    acc = Ct(data, acc.level, acc.scale)
                else:
                    v = self._vec()
                    for m in range(self.M):
                        v[m * self.B] = ly["bias"][m, kk]
                    acc = o.add_plain(acc, self.encode(v, level, bias_scale))
            outs.append(acc)
        return outs

    def _dense_spatial(self, xs, g, H, W, steps, ly, pt_scale, bias_scale, gkeys):
        """Dense layer over the flattened map: for class k, the product of
        every channel with its weight map (w[m][k][c][r][col] at member m's
        grid point (r, col)), summed over channels, plus the bias at slot
        m*block; then the rotation sums over the grid, so slot m*block holds
        the whole dot product."""
        o = self.o
        level = xs[0].level
        K = ly["w"].shape[1]
        outs = []
        for kk in range(K):
            acc = None
            for c, x in enumerate(xs):
                v = self._vec()
                for m in range(self.M):
                    for r in range(H):
                        for col in range(W):
                            v[m * self.B + g * (r * self.W0 + col)] = ly["w"][m, kk, c, r, col]
                term = o.mul_plain(x, self.encode(v, level, pt_scale))
                acc = term if acc is None else o.add(acc, term)
            if ly.get("bias") is not None:
                v = self._vec()
                for m in range(self.M):
                    v[m * self.B] = ly["bias"][m, kk]
                acc = o.add_plain(acc, self.encode(v, level, bias_scale))
            for st in steps:
                acc = o.add(acc, o.rotate(acc, st, gkeys[o.galois_elt(st)]))
            outs.append(acc)
        return outs

    def pool(self, xs, grid, gkeys):
        o = self.o
        g = grid["gap"]
        out = []
        for x in xs:
            y = x
            for st in (g, g * self.W0, g * (self.W0 + 1)):
                y = o.add(y, o.rotate(x, st, gkeys[o.galois_elt(st)]))
            out.append(y)
        return out, dict(gap=2 * g, H=grid["H"] // 2, W=grid["W"] // 2)

    # ------------------------------------------------------------ whole network
    def run(self, sk: SecretKey, inputs, rlk, gkeys, hook=None):
        """inputs: list of channel ciphertexts for ONE image."""
        o = self.o
        tensors = {"x": (inputs, dict(self.input_grid))}
        for ly in self.spec["layers"]:
            xs, grid = tensors[ly["inp"]]
            level, s = xs[0].level, xs[0].scale
            op = ly["op"]
            if op == "conv":
                pt = self._pt_scale(level, s)
                S = s * pt
                outs, ngrid = self.conv(xs, grid, ly, pt, S, gkeys)
                if ly.get("short") is not None:
                    sxs, sgrid = tensors[ly["short"]["inp"]]
                    sxs = [o.mod_drop(c, level) for c in sxs]
                    spt = S / sxs[0].scale
                    souts, _ = self.conv(sxs, sgrid, ly["short"], spt, 1.0, gkeys, with_bias=False)
                    outs = [o.add(a, b) for a, b in zip(outs, souts)]
            elif op == "act":
                outs, ngrid = self.act(xs, ly, rlk, grid), grid
            elif op == "dense":
                pt = self._pt_scale(level, s)
                outs, ngrid = self.dense(xs, grid, ly, pt, s * pt, gkeys), dict(gap=grid["gap"], H=1, W=1)
            elif op == "pool":
                outs, ngrid = self.pool(xs, grid, gkeys)
            else:
                raise ValueError(op)
            if op != "pool" and self._rescale_needed(outs[0].level, outs[0].scale):
                outs = [o.rescale(c) for c in outs]
            tensors[ly["out"]] = (outs, ngrid)
            if hook is not None:
                hook(ly, outs)
        return tensors[self.spec["layers"][-1]["out"]]

    def steps(self):
        """Rotation steps the network needs (for key generation)."""
        st = set()
        grid = dict(self.input_grid)
        grids = {"x": grid}
        for ly in self.spec["layers"]:
            g = grids[ly["inp"]]
            if ly["op"] == "conv":
                half = ly["ksize"] // 2
                for dh in range(-half, half + 1):
                    for dw in range(-half, half + 1):
                        if dh or dw:
                            st.add(g["gap"] * (dh * self.W0 + dw))
                s = ly["stride"]
                grids[ly["out"]] = dict(gap=g["gap"] * s, H=g["H"] // s, W=g["W"] // s)
            elif ly["op"] == "pool":
                st.update([g["gap"], g["gap"] * self.W0, g["gap"] * (self.W0 + 1)])
                grids[ly["out"]] = dict(gap=2 * g["gap"], H=g["H"] // 2, W=g["W"] // 2)
            elif ly["op"] == "dense":
                st.update(g["gap"] * (1 << j) for j in range(int(math.log2(g["W"]))))
                st.update(g["gap"] * self.W0 * (1 << j) for j in range(int(math.log2(g["H"]))))
                grids[ly["out"]] = dict(gap=g["gap"], H=1, W=1)
            else:
                grids[ly["out"]] = g
        if self.spec.get("pack_output"):
            K = self.spec["classes"]
            st.update(-(1 << j) for j in range(max(1, math.ceil(math.log2(K)))))
        return sorted(st)

    # ------------------------------------------------------------ packed output
    def pack_logits(self, cts, gkeys):
        """One image's K class ciphertexts (member m's logit at slot m*block)
        -> one ciphertext with class k at slot m*block + k.  Each class
        ciphertext is multiplied by the mask of the slots m*block, encoded at
        2^(floor(log2 q_l - log2 s) - 7) for its level l and scale s (room for
        the product under q_l), then a binary tree of rotations joins them:
        at depth j, part 2i+1 moves right by 2^j (a rotation by -2^j) and is
        added to part 2i, so after ceil(log2 K) depths class k sits at offset
        k of every member's block."""
        o = self.o
        K = len(cts)
        assert K <= self.B, "classes must fit in a member's block"
        level, s = cts[0].level, cts[0].scale
        ms = 2.0 ** (math.floor(math.log2(float(o.q[level])) - math.log2(s)) - 7)
        v = self._vec()
        for m in range(self.M):
            v[m * self.B] = 1.0
        mask = self.encode(v, level, ms)
        parts = [o.mul_plain(c, mask) for c in cts]
        j = 0
        while len(parts) > 1:
            nxt = []
            for i in range(0, len(parts), 2):
                a = parts[i]
                if i + 1 < len(parts):
                    step = -(1 << j)
                    a = o.add(a, o.rotate(parts[i + 1], step, gkeys[o.galois_elt(step)]))
                nxt.append(a)
            parts = nxt
            j += 1
        return parts[0]
