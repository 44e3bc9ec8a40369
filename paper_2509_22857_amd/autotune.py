"""Autotuner for the evaluator's launch choices.

The library exposes process-wide launch knobs (ckc_tune_set): outputs per
wave and images per workgroup of the convolution contraction, and rotated
inputs per key-switching launch.  Every value gives bit-identical
ciphertexts; only the speed differs with the network's shapes and the batch.
The tuner runs coordinate descent over the knobs: for each knob in turn it
times one whole pass of the network over a representative batch at every
allowed value (the other knobs at their best so far), keeps the fastest, and
checks that the outputs did not change.  The result can be cached in a JSON
file keyed by the workload name.

tune_hoisting picks the key-switching form of each 3x3 convolution (double
or single hoisting) by timing both on the device; that choice is part of the
network description (the two forms differ in the low bits), so it is
returned as marks for the description rather than set in the library.
"""
from __future__ import annotations

import json
import os
import time

from . import ckks

# choices measured on MI355X by this tuner (key: workload / images per pass)
TUNING_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def _pass_time(torch, net, keys, inputs):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, _ = net.run(keys, inputs)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def tune_network(net, keys, inputs, knobs=None, cache: str | None = None, key: str | None = None, log=None,
                 refresh: bool = False, write: bool = True) -> dict:
    """Pick the fastest value of every knob for `net` on the batch `inputs`
    ([n_img][C] ciphertexts); sets the library's knobs and returns
    {knob: value, "timings": {...}}.  With a cache file and key, stored
    choices are applied without timing unless `refresh`; new results are
    written back if `write`."""
    import torch
    knobs = dict(knobs or ckks.TUNE_KNOBS)
    if cache and key and not refresh and os.path.exists(cache):
        with open(cache) as f:
            saved = json.load(f).get(key)
        if saved:
            # knobs the stored choice predates keep the library's default
            for k in knobs:
                if k in saved:
                    ckks.tune_set(k, saved[k])
            return saved
    best = {k: ckks.tune_get(k) for k in knobs}
    timings = {}
    ref = None
    _pass_time(torch, net, keys, inputs)  # warm the tables and scratch arenas
    for k, values in knobs.items():
        scores = {}
        for v in values:
            ckks.tune_set(k, v)
            t, out = _pass_time(torch, net, keys, inputs)
            words = out[0][0].buf.clone()
            if ref is None:
                ref = words
            elif not torch.equal(ref, words):
                raise RuntimeError(f"knob {k}={v} changed the result")
            scores[v] = t
            if log:
                log(f"tune {k}={v}: {t:.3f}s")
        best[k] = min(scores, key=scores.get)
        ckks.tune_set(k, best[k])
        timings[k] = {str(v): round(t, 4) for v, t in scores.items()}
    result = dict(best)
    result["timings"] = timings
    if cache and key and write:
        data = {}
        if os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
        data[key] = result
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return result


def tune_hoisting(net, keys, n_img: int, reps: int = 2, log=None) -> list:
    """The faster key-switching form of every 3x3 convolution of `net`,
    measured: each layer is timed in its current form and in the other one
    (a layer built for the occasion and freed after) on n_img images of
    ciphertexts at the level and scale the planner gives it.  The two forms
    give different low bits (the mark belongs to the network description,
    which both evaluators follow), so the result is a list of marks, one per
    convolution in order (1x1 layers: "double", which they ignore), for
    workloads.nets.set_hoisting.  Replaces the instruction-count model of
    network.choose_hoisting by timings on the device at hand."""
    import torch
    ctx = net.ctx
    marks = []
    for ly, p, ent in zip(net.spec["layers"], net.plans, net.layers):
        if ly["op"] != "conv":
            continue
        if ly["ksize"] == 1:
            marks.append("double")
            continue
        cur = ly.get("hoist", "double")
        other = "single" if cur == "double" else "double"
        lay = net.layouts[ly["inp"]]
        alt = ckks.layer_create_conv(ctx, lay, ly["out_ch"], ly["in_ch"], ly["ksize"], ly["stride"], ly["codebook"],
                                     ly["idx"], ly["bias"], p.level, p.pt_scale, p.bias_scale, hoisting=other)
        ins = [ctx.new_ct(p.level, 2, p.in_scale) for _ in range(n_img * ly["in_ch"])]
        for c in ins:
            c.buf.zero_()
        outs = [ctx.new_ct(p.level) for _ in range(n_img * ly["out_ch"])]
        times = {}
        for form, layer in ((cur, ent["main"]), (other, alt)):
            ckks.eval_conv(ctx, keys, layer, ins, n_img, outs)  # warm the arena
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ckks.eval_conv(ctx, keys, layer, ins, n_img, outs)
            torch.cuda.synchronize()
            times[form] = (time.perf_counter() - t0) / reps
        alt.close()
        del ins, outs
        best = min(times, key=times.get)
        marks.append(best)
        if log:
            log(f"hoisting {ly['name']} (level {p.level}, {ly['in_ch']}->{ly['out_ch']}): "
                f"double {times['double'] * 1e3:.1f} ms, single {times['single'] * 1e3:.1f} ms -> {best}")
    return marks
