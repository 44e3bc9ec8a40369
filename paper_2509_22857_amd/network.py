"""Encrypted CNN evaluation over the C-ABI: level/scale planner and runner.

Planner (tower reuse, Section 4.3): every prime q_i of the chain has a
sublevel lambda(q_i) = round(log_Delta q_i); a ciphertext of scale s has
lambda(s) = round(log_Delta s).  After every multiplicative layer
(convolution, activation, dense) the ciphertext is rescaled iff
lambda(s) > lambda(q_level).  A convolution or dense layer on an input of
scale s at level l encodes its plaintexts at scale (target * q_l) / s so
that its output returns to the target scale after that rescale; its bias
is encoded at s * pt_scale.  A residual shortcut (a 1x1 convolution on the
block input, mod-dropped to the branch's level) encodes at
(s_branch * pt_branch) / s_input so both summands share one scale.  An
activation leaves the level unchanged and squares the scale.

Every homomorphic step runs in libckkscnn.so; this module only sequences the
calls and holds the device buffers (torch tensors).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import ckks


def sublevel(scale: float, delta: float) -> int:
    return int(round(math.log2(scale) / math.log2(delta)))


@dataclass
class LayerPlan:
    op: str
    level: int            # level of the layer's input
    in_scale: float
    pt_scale: float = 1.0
    bias_scale: float = 1.0
    out_scale: float = 1.0   # before the optional rescale
    rescale: bool = False
    short_level: int = -1
    short_pt_scale: float = 1.0


HEADROOM_BITS = 8


def plan_network(spec: dict, q, delta: float, target: float, in_scale: float) -> tuple[list, dict]:
    """Returns (plans per layer, final tensor states {name: (level, scale)})."""
    L = len(q) - 1
    state = {"x": (L, float(in_scale))}
    plans = []

    def after(level, scale):
        if level >= 1 and sublevel(scale, delta) > sublevel(float(q[level]), delta):
            return level - 1, scale / float(q[level]), True
        return level, scale, False

    for ly in spec["layers"]:
        op = ly["op"]
        lv, s = state[ly["inp"]]
        if op in ("conv", "dense"):
            pt = (target * float(q[lv])) / s
            S = s * pt
            p = LayerPlan(op, lv, s, pt_scale=pt, bias_scale=S, out_scale=S)
            if op == "conv" and ly.get("short") is not None:
                ls, ss = state[ly["short"]["inp"]]
                if ls < lv:
                    raise ValueError("shortcut input below the branch level")
                p.short_level = lv
                p.short_pt_scale = S / ss
            nl, ns, p.rescale = after(lv, S)
            state[ly["out"]] = (nl, ns)
        elif op == "act":
            S = (s * s) / float(ly.get("a_absorb", 1.0))
            p = LayerPlan(op, lv, s, out_scale=S)
            nl, ns, p.rescale = after(lv, S)
            state[ly["out"]] = (nl, ns)
        elif op == "pool":
            p = LayerPlan(op, lv, s, out_scale=s)
            state[ly["out"]] = (lv, s)
        else:
            raise ValueError(op)
        if min(state[ly["out"]][0], lv) < 0:
            raise ValueError("chain too short for this network")
        # headroom: values up to 2^(HEADROOM_BITS - 1) in magnitude must stay
        # below half the modulus at the level where the product is formed
        need = math.log2(p.out_scale) + HEADROOM_BITS
        have = sum(math.log2(float(x)) for x in q[:lv + 1])
        if need > have:
            raise ValueError(f"layer {ly['name']}: scale 2^{math.log2(p.out_scale):.1f} leaves less than "
                             f"{HEADROOM_BITS} bits below the modulus at level {lv}; the chain is too short")
        plans.append(p)
    return plans, state


def choose_hoisting(spec: dict, q, n_p: int, delta: float, target: float, in_scale: float,
                     ntt_cost: float = 80.0) -> list[str]:
    """Key-switching form per 3x3 convolution by an operation count, at the
    level the planner gives each layer: double hoisting adds the n_P special
    limbs to every product of the contraction (2 taps O I n_P limb-products),
    single hoisting adds one ModDown per rotated input instead of one per
    output (2 ((taps - 1) I - O) ModDowns of n_P + l + 1 limb transforms,
    each weighed as ntt_cost limb-products; 80 matches per-layer timings of
    both forms on MI355X).  Returns one "single"/"double" per convolution, in
    order (1x1 layers have no rotations: "double", which they ignore); pass
    it to workloads.nets.set_hoisting to mark the network description."""
    plans, _ = plan_network(spec, q, delta, target, in_scale)
    out = []
    for ly, p in zip(spec["layers"], plans):
        if ly["op"] != "conv":
            continue
        taps, I, O = ly["ksize"] ** 2, ly["in_ch"], ly["out_ch"]
        if taps == 1:
            out.append("double")
            continue
        nl = p.level + 1
        extra_products = 2 * taps * O * I * n_p
        saved_moddowns = 2 * ((taps - 1) * I - O) * (n_p + nl) * ntt_cost
        out.append("double" if extra_products < saved_moddowns else "single")
    return out


def input_layout(spec: dict) -> ckks.ckc_layout:
    C, H, W = spec["image"]
    lay = spec["layout"]
    flags = ckks.LAYOUT_SLICE_SHARED if lay.get("slice_shared") else 0
    return ckks.make_layout(lay["block"], lay["row_stride"], 1, H, W, spec["members"], flags)


def image_slots(spec: dict, img: np.ndarray, N: int) -> list[np.ndarray]:
    """Client-side HW packing: channel c -> slot vector with the image copied
    into each member block (all members share the input ciphertexts)."""
    C, H, W = spec["image"]
    B, W0, M = spec["layout"]["block"], spec["layout"]["row_stride"], spec["members"]
    out = []
    for c in range(C):
        v = np.zeros(M * B)
        for m in range(M):
            for r in range(H):
                v[m * B + r * W0: m * B + r * W0 + W] = img[c, r]
        out.append(v)
    return out


def packed_image_slots(spec: dict, imgs: np.ndarray, N: int) -> list[np.ndarray]:
    """Client-side packing of len(imgs) images into one set of ciphertexts
    (a spec from workloads.nets.pack_spec): image p in the member blocks
    p M .. p M + M - 1."""
    C, H, W = spec["image"]
    B, W0 = spec["layout"]["block"], spec["layout"]["row_stride"]
    M, P = spec["packed"]["members"], spec["packed"]["images"]
    assert len(imgs) <= P and M * P * B <= N // 2
    out = []
    for c in range(C):
        v = np.zeros(M * P * B)
        for p, img in enumerate(imgs):
            for m in range(M):
                base = (p * M + m) * B
                for r in range(H):
                    v[base + r * W0: base + r * W0 + W] = img[c, r]
        out.append(v)
    return out


class GpuNetwork:
    """Device-resident layers of one network under one parameter set."""

    def __init__(self, ctx: ckks.Context, spec: dict, delta: float, target: float, in_scale: float):
        self.ctx, self.spec = ctx, spec
        self.delta, self.target, self.in_scale = delta, target, in_scale
        self.plans, self.final = plan_network(spec, ctx.q, delta, target, in_scale)
        self.layers = []
        self.layouts = {"x": input_layout(spec)}
        steps = set()
        for ly, p in zip(spec["layers"], self.plans):
            lay = self.layouts[ly["inp"]]
            entry = {"main": None, "short": None}
            if ly["op"] == "conv":
                entry["main"] = ckks.layer_create_conv(ctx, lay, ly["out_ch"], ly["in_ch"], ly["ksize"], ly["stride"],
                                                       ly["codebook"], ly["idx"], ly["bias"], p.level, p.pt_scale,
                                                       p.bias_scale, hoisting=ly.get("hoist", "double"))
                if ly.get("short") is not None:
                    sh = ly["short"]
                    slay = self.layouts[sh["inp"]]
                    entry["short"] = ckks.layer_create_conv(ctx, slay, sh["out_ch"], sh["in_ch"], sh["ksize"],
                                                            sh["stride"], sh["codebook"], sh["idx"], None,
                                                            p.short_level, p.short_pt_scale, 1.0)
                self.layouts[ly["out"]] = entry["main"].out_layout()
            elif ly["op"] == "act":
                C = ly["b"].shape[1]
                entry["main"] = ckks.layer_create_act(ctx, lay, C, ly["b"], ly["c"], ly.get("a_absorb", 1.0), p.level,
                                                      p.in_scale)
                self.layouts[ly["out"]] = lay
            elif ly["op"] == "dense":
                K, C = ly["w"].shape[1], ly["w"].shape[2]
                entry["main"] = ckks.layer_create_dense(ctx, lay, K, C, ly["w"], ly["bias"], p.level, p.pt_scale,
                                                        p.bias_scale)
                self.layouts[ly["out"]] = entry["main"].out_layout()
            elif ly["op"] == "pool":
                self.layouts[ly["out"]] = ckks.make_layout(lay.block, lay.row_stride, 2 * lay.gap, lay.height // 2,
                                                           lay.width // 2, lay.members, lay.flags)
                steps.update([lay.gap, lay.gap * lay.row_stride, lay.gap * (lay.row_stride + 1)])
            for e in entry.values():
                if e is not None and e.kind in ("conv", "dense"):
                    steps.update(e.steps())
            self.layers.append(entry)
        if spec.get("pack_output"):
            steps.update(-(1 << j) for j in range(max(1, math.ceil(math.log2(spec["classes"])))))
        self.steps = sorted(steps)
        # tensors read by the layers after each layer
        self._later = {}
        lys = self.spec["layers"]
        for i, ly in enumerate(lys):
            later = set()
            for l2 in lys[i + 1:]:
                later.add(l2["inp"])
                if l2.get("short"):
                    later.add(l2["short"]["inp"])
            self._later[ly["name"]] = later

    def device_bytes(self) -> int:
        return sum(e.nbytes() for ent in self.layers for e in ent.values() if e is not None)

    # --------------------------------------------------------- client side
    def encrypt_images(self, keys: ckks.KeyPair, imgs: np.ndarray, stream_base: int = 0):
        """imgs: [n][C][H][W] -> [n][C] ciphertexts at the top level."""
        L = len(self.ctx.q) - 1
        out = []
        for n, img in enumerate(imgs):
            row = []
            for c, v in enumerate(image_slots(self.spec, img, self.ctx.N)):
                pt = self.ctx.encode(v, L, self.in_scale)
                row.append(self.ctx.encrypt(keys, pt, stream_base + n * 4096 + c))
            out.append(row)
        return out

    def encrypt_packed(self, keys: ckks.KeyPair, imgs: np.ndarray, stream_base: int = 0):
        """Packed spec: groups of `images` images -> [n_groups][C] ciphertexts."""
        P = self.spec["packed"]["images"]
        L = len(self.ctx.q) - 1
        out = []
        for g0 in range(0, len(imgs), P):
            row = []
            for c, v in enumerate(packed_image_slots(self.spec, imgs[g0:g0 + P], self.ctx.N)):
                pt = self.ctx.encode(v, L, self.in_scale)
                row.append(self.ctx.encrypt(keys, pt, stream_base + (g0 // P) * 4096 + c))
            out.append(row)
        return out

    def decrypt_logits(self, keys: ckks.KeyPair, cts) -> np.ndarray:
        """One image's class ciphertexts -> logits [M][K] (slot m*block)."""
        B, M = self.spec["layout"]["block"], self.spec["members"]
        res = []
        for ct in cts:
            z = self.ctx.decode(self.ctx.decrypt(keys, ct), M * B)
            res.append([z[m * B] for m in range(M)])
        return np.array(res).T

    def pack_logits(self, keys: ckks.KeyPair, cts, stream=None):
        """One image's K class ciphertexts -> one ciphertext with class k at
        slot m*block + k (needs "pack_output" in the network description, for
        the keys of the steps -2^j).  Each class ciphertext is multiplied by
        the mask of the slots m*block, encoded at 2^(floor(log2 q_l - log2 s)
        - 7) for its level l and scale s, then a binary tree of rotations
        joins them: at depth j, part 2i+1 moves right by 2^j and is added to
        part 2i."""
        ctx = self.ctx
        K, B, M = len(cts), self.spec["layout"]["block"], self.spec["members"]
        if K > B:
            raise ValueError("classes must fit in a member's block")
        level, s = cts[0].level, cts[0].scale
        ms = 2.0 ** (math.floor(math.log2(float(ctx.q[level])) - math.log2(s)) - 7)
        v = np.zeros(ctx.N // 2)
        v[[m * B for m in range(M)]] = 1.0
        mask = ctx.encode(v, level, ms, stream=stream)
        parts = [ctx.mul_plain(c, mask, stream=stream) for c in cts]
        j = 0
        while len(parts) > 1:
            nxt = []
            for i in range(0, len(parts), 2):
                a = parts[i]
                if i + 1 < len(parts):
                    r = ctx.rotate(keys, parts[i + 1], [-(1 << j)], stream=stream)[0]
                    a = ctx.add(a, r, stream=stream)
                nxt.append(a)
            parts = nxt
            j += 1
        return parts[0]

    def decrypt_packed_logits(self, keys: ckks.KeyPair, ct) -> np.ndarray:
        """A packed logits ciphertext -> [M][K] (class k of member m at slot m*block + k)."""
        B, M, K = self.spec["layout"]["block"], self.spec["members"], self.spec["classes"]
        z = self.ctx.decode(self.ctx.decrypt(keys, ct), M * B)
        return np.array([[z[m * B + k] for k in range(K)] for m in range(M)])

    def decrypt_grid(self, keys: ckks.KeyPair, ct, layout) -> np.ndarray:
        """One channel ciphertext -> values on the valid grid [M][H][W]."""
        L = layout
        z = self.ctx.decode(self.ctx.decrypt(keys, ct), L.members * L.block)
        out = np.zeros((L.members, L.height, L.width))
        for m in range(L.members):
            for r in range(L.height):
                for c in range(L.width):
                    out[m, r, c] = z[m * L.block + L.gap * (r * L.row_stride + c)]
        return out

    # --------------------------------------------------------- server side
    def run(self, keys: ckks.KeyPair, inputs, stream=None, keep=False, hook=None, images_per_pass=None):
        """inputs: [n_img][C] ciphertexts -> ([n_img][K or C] ciphertexts, tensors).

        Every tensor of the network is evaluated for all images of a pass
        before the next layer starts; images_per_pass bounds the live
        ciphertexts (a pass of 16 ResNet-20 images already fills every key
        switching launch with 64 ciphertexts).  With several passes the
        returned tensors are those of the last pass."""
        if images_per_pass and len(inputs) > images_per_pass:
            outs, tensors = [], None
            for i in range(0, len(inputs), images_per_pass):
                ki = keys.slice(i, i + images_per_pass) if isinstance(keys, ckks.KeyGroup) else keys
                o, tensors = self.run(ki, inputs[i:i + images_per_pass], stream, keep, hook)
                outs.extend(o)
            return outs, tensors
        it = self.stages(keys, inputs, stream, keep, hook)
        while True:
            try:
                next(it)
            except StopIteration as stop:
                return stop.value

    def stages(self, keys: ckks.KeyPair, inputs, stream=None, keep=False, hook=None):
        """Generator form of run(): each step enqueues one layer (all images)
        on `stream` and yields the layer's name; the generator's return value
        is run()'s.  Buffers of a step are allocated on `stream`, so steps of
        different generators may interleave on different streams."""
        import torch
        ctx = self.ctx
        n_img = len(inputs)
        tensors = {"x": [c for row in inputs for c in row]}
        scope = torch.cuda.stream(stream) if stream is not None else _NoScope()
        for ly, p, ent in zip(self.spec["layers"], self.plans, self.layers):
            with scope:
                outs = self._layer(keys, ly, p, ent, tensors, n_img, stream)
            tensors[ly["out"]] = outs
            if hook is not None:
                hook(ly, outs)
            if not keep:
                # drop tensors no later layer reads
                for name in list(tensors):
                    if name not in self._later[ly["name"]] and name != ly["out"]:
                        del tensors[name]
            yield ly["name"]
        last = self.spec["layers"][-1]["out"]
        flat = tensors[last]
        per = len(flat) // n_img
        return [flat[i * per:(i + 1) * per] for i in range(n_img)], tensors

    def _layer(self, keys, ly, p, ent, tensors, n_img, stream):
        ctx = self.ctx
        xin = tensors[ly["inp"]]
        op = ly["op"]
        if op == "conv":
            O = ly["out_ch"]
            outs = [ctx.new_ct(p.level) for _ in range(n_img * O)]
            ckks.eval_conv(ctx, keys, ent["main"], xin, n_img, outs, stream)
            if ent["short"] is not None:
                xs = tensors[ly["short"]["inp"]]
                if xs[0].level != p.short_level:
                    xs = [ctx.mod_drop(c, p.short_level, stream=stream) for c in xs]
                souts = [ctx.new_ct(p.short_level) for _ in range(n_img * O)]
                ckks.eval_conv(ctx, keys, ent["short"], xs, n_img, souts, stream)
                ckks.add_many(ctx, outs, souts, outs, stream)
        elif op == "act":
            outs = [ctx.new_ct(p.level) for _ in range(len(xin))]
            ckks.eval_quad_act(ctx, keys, ent["main"], xin, n_img, outs, stream)
        elif op == "dense":
            K = ly["w"].shape[1]
            outs = [ctx.new_ct(p.level) for _ in range(n_img * K)]
            ckks.eval_dense(ctx, keys, ent["main"], xin, n_img, outs, stream)
        elif op == "pool":
            outs = [ctx.new_ct(p.level) for _ in range(len(xin))]
            ckks.eval_avgpool2(ctx, keys, self.layouts[ly["inp"]], xin, outs, stream)
        else:
            raise ValueError(f"unknown layer op {op}")
        if p.rescale:
            r = [ctx.new_ct(p.level - 1) for _ in range(len(outs))]
            ckks.rescale_many(ctx, outs, r, stream)
            outs = r
        return outs

    def native_plan(self) -> "ckks.Plan":
        """The network as a program for the library's native runner (the same
        layer calls, rescales and residual additions as stages())."""
        import json
        handles = []

        def idx(layer):
            handles.append(layer)
            return len(handles) - 1

        count_of = {"x": self.spec["image"][0]}
        steps = []
        for ly, p, ent in zip(self.spec["layers"], self.plans, self.layers):
            op = ly["op"]
            st = {"op": op, "in": ly["inp"], "out": ly["out"], "level": p.level, "rescale": int(bool(p.rescale))}
            if op == "conv":
                st["count"], st["layer"] = ly["out_ch"], idx(ent["main"])
                if ent["short"] is not None:
                    st["short"] = {"layer": idx(ent["short"]), "in": ly["short"]["inp"], "level": p.short_level}
            elif op == "act":
                st["count"], st["layer"] = count_of[ly["inp"]], idx(ent["main"])
            elif op == "dense":
                st["count"], st["layer"] = ly["w"].shape[1], idx(ent["main"])
            elif op == "pool":
                lay = self.layouts[ly["inp"]]
                st["count"] = count_of[ly["inp"]]
                st["layout"] = {k: int(getattr(lay, k)) for k in ("block", "row_stride", "gap", "height", "width",
                                                                   "members", "flags")}
            else:
                raise ValueError(f"unknown layer op {op}")
            count_of[ly["out"]] = st["count"]
            steps.append(st)
        program = {"input": {"name": "x", "count": self.spec["image"][0], "level": len(self.ctx.q) - 1},
                   "output": self.spec["layers"][-1]["out"], "steps": steps}
        return ckks.Plan(self.ctx, json.dumps(program), handles)

    def working_set_bytes(self, n_img: int) -> int:
        """Upper estimate of the device bytes one pass of n_img images holds:
        the most live tensors around any layer plus the largest scratch of any
        layer (rotated inputs, a 3x3 layer's outputs over Q_l and P, digits
        and key-switching buffers of one batch of 64), which the stream's
        scratch arena keeps for the whole pass."""
        held, scratch = self._memory(n_img)
        return int(1.1 * (held + scratch))

    def scratch_bytes(self, n_img: int) -> int:
        """Upper estimate of the largest scratch one call of a pass of n_img
        images takes (the size to reserve for the stream's arena)."""
        return int(1.1 * self._memory(n_img)[1])

    def _memory(self, n_img: int):
        N = self.ctx.N
        np_ = len(self.ctx.p)
        ct = lambda level, npoly=2: 8 * npoly * (level + 1) * N
        level_of = {"x": len(self.ctx.q) - 1}
        count_of = {"x": self.spec["image"][0]}
        max_held = max_scratch = 0
        live = {"x"}
        for ly, p in zip(self.spec["layers"], self.plans):
            lvl = p.level
            out_lvl = p.level - 1 if p.rescale else p.level
            if ly["op"] == "conv":
                cnt = ly["out_ch"]
            elif ly["op"] == "dense":
                cnt = ly["w"].shape[1]
            else:
                cnt = count_of[ly["inp"]]
            level_of[ly["out"]], count_of[ly["out"]] = out_lvl, cnt
            held = sum(n_img * count_of[t] * ct(level_of[t]) for t in live)
            held += n_img * cnt * ct(lvl) * (2 if p.rescale else 1)
            nl, nt = lvl + 1, lvl + 1 + np_
            dnum = -(-nl // self.ctx.alpha)
            ks = 64 * 8 * N * (dnum * nt + 2 * nl + 2 * np_ + 2 * nl + nl)
            if ly["op"] == "conv":
                # rotated inputs of one input-channel chunk (at most 64) for a
                # group of images; a 3x3 layer keeps them, and its outputs
                # before ModDown, over Q_l and P
                I, taps = ly["in_ch"], ly["ksize"] ** 2
                ich = min(I, 64)
                nimg = min(max(4, 64 // ich), n_img)
                ext = ly["ksize"] > 1 and ly.get("hoist", "double") == "double"
                cte = 8 * 2 * (nt if ext else nl) * N
                scratch = nimg * ich * taps * cte + (nimg * cnt * cte if ext else 0) + ks
                if ly.get("short") is not None:
                    held += n_img * cnt * ct(p.short_level)
            elif ly["op"] == "act":
                scratch = 64 * ct(lvl, 3) + ks
            else:
                scratch = 2 * n_img * cnt * ct(lvl) + ks
            max_held, max_scratch = max(max_held, held), max(max_scratch, scratch)
            live = set(self._later[ly["name"]]) | {ly["out"]}
            live = {t for t in live if t in level_of}
        return max_held, max_scratch


class _NoScope:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False
