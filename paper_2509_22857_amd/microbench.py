"""Kernel microbenchmark of the evaluator's operations at N = 2^16.

Parameters: 24 RNS primes of 50 bits, 3 special primes of 50 bits, three
primes per key-switching digit (dnum = 8 at the top level).  A batch of
random ciphertexts (uniform residues, seeded) at the top level goes through
each operation separately:

  ntt_fwd / ntt_inv   every limb of every polynomial, in place
  rotate              hoisted rotations by {0, +-1, +-31, +-32, +-33}, the
                      batch in one call (keys reused across it), and one
                      ciphertext per call (every call streams the keys)
  mac                 out[i] = sum over the 9 rotations of pt_t * Rot_t(ct_i)
  mul_relin           Relin(ct_i * ct_i)
  rescale             drop the top prime

Each operation is timed with events on the stream it runs on; with launch
profiling on, the library's per-kernel-class times and algorithmic bytes
give the HBM fraction of the key-switching kernels.
"""
from __future__ import annotations

import time

import numpy as np

from . import ckks
from workloads import params

STEPS = (0, 1, -1, 32, -32, 33, -33, 31, -31)
HBM_PEAK_GBS = 8000.0
KS_CLASSES = ("ntt_fwd", "ntt_inv", "bconv", "kip", "moddown")


def _random_cts(ctx, torch, n, level, seed):
    """n 2-polynomial ciphertexts with uniform residues (seeded, generated on the device)."""
    g = torch.Generator(device=ctx.device)
    g.manual_seed(seed)
    nl = level + 1
    out = []
    for _ in range(n):
        ct = ctx.new_ct(level, 2, 2.0 ** 40)
        v = ct.buf.view(2, nl, ctx.N)
        for li in range(nl):
            v[:, li].random_(0, ctx.q[li], generator=g)
        out.append(ct)
    return out


def _random_pts(ctx, torch, n, level, seed):
    g = torch.Generator(device=ctx.device)
    g.manual_seed(seed)
    out = []
    for _ in range(n):
        pt = ctx.new_pt(level, 2.0 ** 40)
        v = pt.buf.view(level + 1, ctx.N)
        for li in range(level + 1):
            v[li].random_(0, ctx.q[li], generator=g)
        out.append(pt)
    return out


def _profile(ckks, torch, fn):
    """Per-kernel-class time and algorithmic-byte rate of one call of fn, and
    the HBM fraction of its key-switching kernels taken together."""
    ckks.prof_enable(True)
    fn()
    torch.cuda.synchronize()
    prof = {k: ckks.prof_query(k) for k in KS_CLASSES}
    ckks.prof_enable(False)
    ks_ms = sum(p["ms"] for p in prof.values())
    ks_bytes = sum(p["bytes"] for p in prof.values())
    kern = {k: {"ms": round(p["ms"], 3), "launches": p["launches"],
                "GBs": round(p["bytes"] / (p["ms"] * 1e-3) / 1e9, 1) if p["ms"] else 0.0}
            for k, p in prof.items()}
    frac = ks_bytes / (ks_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if ks_ms else 0.0
    return kern, frac


class _Timer:
    def __init__(self, torch):
        self.torch = torch

    def __call__(self, fn, reps):
        torch = self.torch
        s = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(reps):
            fn()
        b.record(s)
        b.synchronize()
        return a.elapsed_time(b) / reps


def run(batch: int = 64, reps: int = 3, seed: int = 7, log=print) -> dict:
    import torch
    ps = params.micro()
    ctx = ckks.Context.from_params(ps)
    N, W = ctx.N, 8.0 * ctx.N
    level = len(ps.q) - 1
    nl, npr = level + 1, len(ps.p)
    nt = nl + npr
    dnum = -(-nl // ps.alpha)
    t0 = time.time()
    keys = ctx.keygen(seed, [s for s in STEPS if s])
    key_words = dnum * 2 * (len(ps.q) + npr) * N
    cts = _random_cts(ctx, torch, batch, level, seed + 1)
    pts = _random_pts(ctx, torch, len(STEPS), level, seed + 2)
    torch.cuda.synchronize()
    log(f"micro: keys + {batch} ciphertexts ready in {time.time() - t0:.1f}s "
        f"(evk {keys.evk_bytes() / 2**30:.2f} GiB)")
    timer = _Timer(torch)
    res = {}

    def record(name, ms, bytes_, extra=None):
        gbs = bytes_ / (ms * 1e-3) / 1e9
        r = {"ms": round(ms, 3), "us_per_ct": round(1e3 * ms / batch, 2), "GBs": round(gbs, 1),
             "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        if extra:
            r.update(extra)
        res[name] = r
        log(f"  {name:10s} {ms:9.3f} ms/batch  {r['us_per_ct']:9.2f} us/ct  {gbs:8.1f} GB/s  "
            f"({100 * gbs / HBM_PEAK_GBS:.1f}% HBM)" + (f"  {extra}" if extra else ""))

    # one contiguous buffer for the NTT rows: batch x 2 polynomials x nl limbs
    big = torch.cat([c.buf for c in cts])
    for inv in (0, 1):
        name = "ntt_inv" if inv else "ntt_fwd"
        ctx.ntt(big, 2 * batch, nl, bool(inv))
        ms = timer(lambda: ctx.ntt(big, 2 * batch, nl, bool(inv)), reps)
        record(name, ms, 2.0 * W * 2 * nl * batch)
    del big

    outs = [ctx.new_ct(level, 2) for _ in range(batch * len(STEPS))]
    nz = sum(1 for s in STEPS if s)

    def rot():
        ckks.rotate_many(ctx, keys, cts, STEPS, outs)

    rot()
    ms = timer(rot, reps)
    kern, ks_frac = _profile(ckks, torch, rot)
    # op-level algorithmic bytes: inputs, every Galois key once per 64 inputs, outputs
    key_bytes = 8.0 * key_words
    rot_bytes = W * 2 * nl * batch * (1 + len(STEPS)) + nz * key_bytes * -(-batch // 64)
    record("rotate", ms, rot_bytes, {"ks_kernel_hbm_frac": round(ks_frac, 4)})
    res["rotate"]["kernels"] = kern
    res["key_switch_hbm_frac"] = round(ks_frac, 4)

    # the same hoisted group one ciphertext per call (no key reuse across
    # ciphertexts: every call streams all eight Galois keys -- the regime of a
    # single client's request)
    n1 = min(8, batch)

    def rot1():
        for i in range(n1):
            ckks.rotate_many(ctx, keys, cts[i:i + 1], STEPS, outs[i * len(STEPS):(i + 1) * len(STEPS)])

    rot1()
    ms1 = timer(rot1, reps)
    kern1, ks_frac1 = _profile(ckks, torch, rot1)
    rot1_bytes = W * 2 * nl * n1 * (1 + len(STEPS)) + nz * key_bytes * n1
    r = {"ms": round(ms1, 3), "us_per_ct": round(1e3 * ms1 / n1, 2),
         "GBs": round(rot1_bytes / (ms1 * 1e-3) / 1e9, 1),
         "hbm_frac": round(rot1_bytes / (ms1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
         "ks_kernel_hbm_frac": round(ks_frac1, 4), "kernels": kern1, "ciphertexts": n1}
    res["rotate_one_at_a_time"] = r
    log(f"  rotate 1x  {ms1:9.3f} ms/{n1} cts {r['us_per_ct']:9.2f} us/ct  {r['GBs']:8.1f} GB/s  "
        f"({100 * r['hbm_frac']:.1f}% HBM, key-switch kernels {100 * ks_frac1:.1f}%)")

    macs = [ctx.new_ct(level, 2) for _ in range(batch)]
    ckks.mac_plain_many(ctx, outs, pts, macs)
    ms = timer(lambda: ckks.mac_plain_many(ctx, outs, pts, macs), reps)
    record("mac", ms, W * nl * (2 * batch * len(STEPS) + len(STEPS) + 2 * batch))
    del outs

    sq = [ctx.new_ct(level, 2) for _ in range(batch)]

    def mr():
        ckks.mul_relin_many(ctx, keys, cts, cts, sq)

    mr()
    ms = timer(mr, reps)
    kern, frac = _profile(ckks, torch, mr)
    record("mul_relin", ms, W * 4 * nl * batch + key_bytes * -(-batch // 64), {"ks_kernel_hbm_frac": round(frac, 4)})
    res["mul_relin"]["kernels"] = kern

    rs = [ctx.new_ct(level - 1, 2) for _ in range(batch)]
    for c in cts:
        c.scale = 2.0 ** 40
    ckks.rescale_many(ctx, cts, rs)
    ms = timer(lambda: ckks.rescale_many(ctx, cts, rs), reps)
    record("rescale", ms, W * (2 * nl + 2 * (nl - 1)) * batch)
    res["config"] = {"logN": ps.logN, "n_q": len(ps.q), "n_p": npr, "alpha": ps.alpha, "dnum": dnum,
                     "batch": batch, "level": level, "steps": list(STEPS)}
    return res
