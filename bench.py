"""Benchmark: encrypted images/s of a ResNet-20-style ensemble at N = 2^16.

One step = the whole encrypted network (every convolution, activation,
rescale and the dense layer) over one batch of client-encrypted images that
are already resident in HBM.  The same kernels also run one image at a time
("plain") for the batched-vs-plain comparison.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

HBM_PEAK_GBS = 8000.0
MODMUL_PEAK_T = 256 * 64 * 2.4e9 / 4 / 1e12   # 9.83 T 64-bit modular products/s
MUL_BOUND = ("conv_contract", "dense_mac", "mac_plain")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# device code whose change invalidates a kernel class's measured HBM traffic:
# (file, first line of the region, text that ends it) — None: the whole file
TRAFFIC_SOURCES = {"conv_contract": (("paper_2509_22857_amd/csrc/layers.hip", "constexpr int kMaxCentLds",
                                      "using ConvFn"),
                                     ("paper_2509_22857_amd/csrc/modarith.h", None, None))}


def kernel_source_hash(cls):
    h = hashlib.sha256()
    for rel, start, end in TRAFFIC_SOURCES.get(cls, ()):
        with open(os.path.join(ROOT, rel), "rb") as f:
            text = f.read()
        if start is not None:
            a = text.index(start.encode())
            text = text[a:text.index(end.encode(), a)]
        h.update(text)
    return h.hexdigest()[:16]


def measured_traffic(cls, workload_key):
    """HBM bytes per launch of kernel class `cls` from its committed counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    same counter reads for a copy of known size in the same run), or None
    when there is no summary, it was taken for another workload or launch
    choice, or the kernel's sources have changed since."""
    path = os.path.join(ROOT, "profiles", f"{cls}_traffic.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            k, sep, v = line.partition(": ")
            if sep and k.strip().replace("_", "").isalnum():
                rec[k.strip()] = v.strip()
    if rec.get("sources_sha256_16") != kernel_source_hash(cls) or rec.get("workload_key") != workload_key:
        return None
    return {"bytes_per_launch": float(rec["traffic_bytes_per_launch"]),
            "fetch_bytes_per_launch": float(rec["fetch_bytes_per_launch"]),
            "write_bytes_per_launch": float(rec["write_bytes_per_launch"])}


def calibration_copy(torch):
    """One device copy of a known size (1 GiB read + 1 GiB written): the
    reference kernel for scaling hardware byte counters (FETCH_SIZE,
    WRITE_SIZE) of the evaluator's kernels in the same run."""
    src = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def run_packed(args):
    """Slot packing, a separate labelled row (not the headline): args.pack
    images share every ciphertext (image p in member blocks p M .. p M + M - 1
    of the same network), so one pass over the ciphertexts serves pack images.
    Prints its own JSON line."""
    import torch
    from paper_2509_22857_amd.autotune import tune_network, TUNING_FILE
    from paper_2509_22857_amd.ckks import Context
    from paper_2509_22857_amd.network import GpuNetwork
    from oracle.forward import forward
    from workloads import gen, nets
    P = args.pack
    t0 = time.time()
    ps, spec = build_workload(args)
    pspec = nets.pack_spec(spec, P)
    M, B = spec["members"], spec["layout"]["block"]
    if M * P * B > (1 << ps.logN) // 2:
        log(f"{P} images x {M} members x {B} slots do not fit N/2 slots")
        sys.exit(2)
    ctx = Context.from_params(ps)
    delta = 2.0 ** ps.delta_log2
    net = GpuNetwork(ctx, pspec, delta, delta, delta)
    keys = ctx.keygen(12345, net.steps)
    torch.cuda.synchronize()
    log(f"packed: {P} images x {M} members per ciphertext, set-up {time.time() - t0:.1f}s")
    n_img = args.batch
    imgs = gen.images(777, n_img, *spec["image"])
    groups = net.encrypt_packed(keys, imgs, stream_base=1 << 20)
    torch.cuda.synchronize()
    if args.tune != "off":
        tune_network(net, keys, groups[: min(len(groups), args.images_per_pass)], cache=TUNING_FILE,
                     key=f"resnet20_ensemble_N65536/{min(len(groups), args.images_per_pass)}", write=False)
    for _ in range(args.warmup):
        net.run(keys, groups, images_per_pass=args.images_per_pass)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        out, _ = net.run(keys, groups, images_per_pass=args.images_per_pass)
    ev1.record(stream)
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) / 1e3 / args.steps
    ips = n_img / sec
    log(f"packed batched: {sec:.2f}s per step of {n_img} images ({len(groups)} ciphertext groups) -> {ips:.3f} images/s")
    max_err, agree, nchk = 0.0, 0, 0
    for g in range(min(len(groups), max(1, args.check // P))):
        got = net.decrypt_logits(keys, out[g]).reshape(P, M, -1)
        for p in range(P):
            i = g * P + p
            if i >= n_img:
                break
            ref = forward(spec, imgs[i])
            max_err = max(max_err, float(np.max(np.abs(got[p] - ref))))
            agree += int(got[p].mean(0).argmax() == ref.mean(0).argmax())
            nchk += 1
    log(f"packed logits vs FP64: max abs err {max_err:.2e}, top-1 agree {agree}/{nchk}")
    print(json.dumps({
        "metric": "encrypted images/s (ResNet-20-style ensemble, N=2^16, slot-packed row, not the headline)",
        "value": round(ips, 4), "unit": "images/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 1), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "resnet20_ensemble_N65536_slot_packed", "images_per_ciphertext": P,
                   "members": M, "images_per_step": n_img, "ciphertext_groups_per_pass": args.images_per_pass},
        "accuracy": {"max_abs_logit_err": max_err, "top1_agree": f"{agree}/{nchk}"},
        "roofline": None, "cpu_baseline": None}))


def workload_key(args, tuned):
    knobs = {k: v for k, v in (tuned or {}).items() if k != "timings"}
    return (f"{args.workload}/{args.layout}/batch{args.batch}/pass{args.images_per_pass}/" +
            json.dumps(knobs, sort_keys=True))


VGG_HOISTING = ["single", "double", "double", "double", "single"]


def build_workload(args):
    """Parameters and network of the workload.  Layout: slice-shared (Section
    5.2: one plaintext per kernel column and centroid, vertical padding from
    zero rows, so each 32x32 image takes a block of 2048 slots, 64 rows of 32)
    unless --layout taps (one plaintext per tap and centroid, blocks of 1024
    slots) or slot packing, which needs the smaller blocks."""
    from workloads import nets
    from workloads.params import resnet20_tower
    shared = getattr(args, "layout", "slice") == "slice" and getattr(args, "pack", 1) == 1
    if args.workload == "vgg":
        # VGG-style: 3->64, 64->64, pool, 64->128, 128->128, pool, 128->256,
        # dense over the flattened 256 x 8 x 8 map to 10 classes; k = 16.
        # Per-layer key-switching form: what network.choose_hoisting picks for
        # this network and chain (a test keeps the two in step): the first
        # layer (3 inputs, 64 outputs) and the last (level 2: three Q limbs,
        # to which the three P limbs would add as many again) single-hoisted
        ps = resnet20_tower(levels=6)
        spec = nets.vgg_spec(seed=0, calib=8, hoist=VGG_HOISTING, dense="flatten")
    else:
        ps = resnet20_tower()
        spec = nets.resnet_spec(seed=0, members=4, widths=(16, 32, 64), blocks=3, classes=100, image=(3, 32, 32),
                                k=64, calib=8)
    if shared:
        spec["layout"]["block"] = 2048
        spec["layout"]["slice_shared"] = True
    return ps, spec


def _fit3(xs, ys):
    """Quadratic through three points (x, y), as a callable."""
    c = np.polyfit(np.array(xs, dtype=float), np.array(ys, dtype=float), 2)
    return lambda x: float(max(np.polyval(c, x), min(ys)))


def cpu_baseline(ps, spec, gpu_products_per_image=None):
    """The oracle as it stands, timed on this host per operation class on the
    workload's own chain, and composed into one image from the operation
    counts of the oracle's evaluation of the network (its level schedule
    gives every layer's level).  Timed classes: the key switch with and
    without ModDown (the rotation and the extended rotation of a double-
    hoisted convolution) and ModDown alone at three levels spanning the
    schedule (a quadratic in the limb count between them), rescale at the
    same levels, and per limb the negacyclic product (the oracle multiplies
    in coefficient form), the automorphism, the multiplication by P and the
    modular addition.  No GPU time enters the figure."""
    import platform
    from oracle.ckks import Ct, Oracle
    from oracle.network import OracleNetwork
    from workloads import gen
    o = Oracle.from_params(ps)
    D = 2.0 ** ps.delta_log2
    net = OracleNetwork(o, spec, D, D, D)
    sch = net.schedule()
    t_all = time.time()
    sk = o.secret_key(1)
    g = o.galois_elt(1)
    gk = o.galois_key(sk, g)
    lv_used = sorted({s["level_in"] for s in sch})
    levels = sorted({lv_used[0], lv_used[len(lv_used) // 2], lv_used[-1]})
    N = ps.N
    np_ = len(ps.p)
    ks, ks_ext, mdown, resc = {}, {}, {}, {}
    for lv in levels:
        d = gen.random_ct(3, ps.q, lv, N)
        a = time.time(); o.keyswitch(d[1], lv, gk, g); ks[lv] = time.time() - a
        a = time.time(); o.keyswitch_ext(d[1], lv, gk, g); ks_ext[lv] = time.time() - a
        x = gen.random_limbs(5, list(ps.q[:lv + 1]) + list(ps.p), N)
        a = time.time(); o.moddown(x, lv); mdown[lv] = time.time() - a
        a = time.time(); o.rescale(Ct(d, lv, D * D)); resc[lv] = time.time() - a
    x1 = [lv + 1 for lv in levels]
    if len(levels) < 3:
        x1 = x1 + [x1[-1] + 1] * (3 - len(levels))
    f_ks = _fit3(x1, [ks[lv] for lv in levels] + [ks[levels[-1]]] * (3 - len(levels)))
    f_ext = _fit3(x1, [ks_ext[lv] for lv in levels] + [ks_ext[levels[-1]]] * (3 - len(levels)))
    f_md = _fit3(x1, [mdown[lv] for lv in levels] + [mdown[levels[-1]]] * (3 - len(levels)))
    f_rs = _fit3(x1, [resc[lv] for lv in levels] + [resc[levels[-1]]] * (3 - len(levels)))
    a_ = gen.random_ct(9, ps.q, 0, N)[0, 0]
    b_ = gen.random_ct(10, ps.q, 0, N)[0, 0]
    reps = 8
    a = time.time()
    for _ in range(reps):
        o.polymul(a_, b_, 0)
    t_mul = (time.time() - a) / reps
    a = time.time()
    for _ in range(reps):
        o.automorphism(a_, g, 0)
    t_aut = (time.time() - a) / reps
    P0 = 1
    for pk in ps.p:
        P0 = P0 * pk % ps.q[0]
    a = time.time()
    for _ in range(reps):
        ((a_.astype(object) * P0) % ps.q[0]).astype(np.uint64)
    t_P = (time.time() - a) / reps
    q0 = np.uint64(ps.q[0])
    a = time.time()
    for _ in range(reps):
        o._add(a_, b_, q0)
    t_add = (time.time() - a) / reps
    t_meas = time.time() - t_all

    # the oracle's operations per image, layer by layer (OracleNetwork.run)
    cnt = {"ks": 0.0, "ks_ext": 0.0, "moddown": 0.0, "rescale": 0.0, "limb_mul": 0.0, "limb_aut": 0.0,
           "limb_P": 0.0, "limb_add": 0.0}
    sec = {k: 0.0 for k in cnt}
    per_level = {"ks": f_ks, "ks_ext": f_ext, "moddown": f_md, "rescale": f_rs}
    per_limb = {"limb_mul": t_mul, "limb_aut": t_aut, "limb_P": t_P, "limb_add": t_add}

    def add(kind, n, lv=None):
        cnt[kind] += n
        sec[kind] += n * (per_level[kind](lv + 1) if kind in per_level else per_limb[kind])

    ch = {"x": spec["image"][0]}
    products = 0.0
    for ly, st in zip(spec["layers"], sch):
        lv = st["level_in"]
        nl, nt = lv + 1, lv + 1 + np_
        op = ly["op"]
        if op == "conv":
            I, O, T = ly["in_ch"], ly["out_ch"], ly["ksize"] ** 2
            ch[ly["out"]] = O
            if T == 1:
                add("limb_mul", O * I * 2 * nl); add("limb_add", O * I * 2 * nl)
                products += O * I * 2 * nl
            elif ly.get("hoist", "double") == "single":
                add("ks", I * (T - 1), lv); add("limb_aut", I * (T - 1) * nl); add("limb_add", I * (T - 1) * nl)
                add("limb_mul", O * I * T * 2 * nl); add("limb_add", O * I * T * 2 * nl)
                products += O * I * T * 2 * nl
            else:
                add("ks_ext", I * (T - 1), lv)
                add("limb_aut", I * (T - 1) * nl); add("limb_P", I * (T - 1) * nl + I * 2 * nl)
                add("limb_add", I * (T - 1) * nl)
                add("limb_mul", O * I * T * 2 * nt); add("limb_add", O * I * T * 2 * nt)
                add("moddown", 2 * O, lv)
                products += O * I * T * 2 * nt
            if ly.get("bias") is not None:
                add("limb_add", O * nl)
            if ly.get("short") is not None:
                sh = ly["short"]
                add("limb_mul", O * sh["in_ch"] * 2 * nl); add("limb_add", O * sh["in_ch"] * 2 * nl + O * 2 * nl)
                products += O * sh["in_ch"] * 2 * nl
        elif op == "act":
            C = ch[ly["inp"]]
            ch[ly["out"]] = C
            add("limb_mul", C * 4 * nl); add("limb_add", C * (1 + 2 + 2) * nl); add("ks", C, lv)
        elif op == "dense":
            C, K = ch[ly["inp"]], ly["w"].shape[1]
            ch[ly["out"]] = K
            nrot = int(math.log2(spec["image"][1])) + int(math.log2(spec["image"][2]))
            add("ks", C * nrot, lv); add("limb_aut", C * nrot * nl); add("limb_add", C * nrot * 3 * nl)
            add("limb_mul", K * C * 2 * nl); add("limb_add", K * C * 2 * nl + K * nl)
            products += K * C * 2 * nl
        elif op == "pool":
            C = ch[ly["inp"]]
            ch[ly["out"]] = C
            add("ks", 3 * C, lv); add("limb_aut", 3 * C * nl); add("limb_add", 3 * C * 3 * nl)
        if st["rescale"]:
            add("rescale", ch[ly["out"]], lv)
    sec_per_image = sum(sec.values())
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        model = platform.processor() or "unknown"
    parts = ", ".join(f"{k} {cnt[k]:.4g} x -> {sec[k]:.1f} s" for k in cnt)
    unit = (f"key switch {ks[levels[-1]]:.2f} s / extended {ks_ext[levels[-1]]:.2f} s / ModDown "
            f"{mdown[levels[-1]]:.3f} s / rescale {resc[levels[-1]]:.3f} s at level {levels[-1]} "
            f"(also timed at levels {levels[:-1]}); per limb: product {1e3 * t_mul:.2f} ms, automorphism "
            f"{1e3 * t_aut:.2f} ms, times P {1e3 * t_P:.2f} ms, addition {1e3 * t_add:.3f} ms")
    chk = ""
    if gpu_products_per_image:
        chk = (f"; limb-products of the convolutions and dense layer: oracle {products:.4g} per image, "
               f"GPU counter {gpu_products_per_image / N:.4g} (the GPU skips the identity tap on the P limbs)")
    return {"value": 1.0 / sec_per_image, "unit": "images/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle (single-threaded C + numpy) on {model}, nproc {os.cpu_count()}; {t_meas:.1f} s of "
                       f"timing: {unit}; composed per image from the oracle's operation counts: {parts}; "
                       f"{sec_per_image:.0f} s per image{chk}")}


def run_chw(args):
    """The CHW layout (every channel of an image in one ciphertext), a
    separate labelled row: 32 channels of 32 x 32 fill the 2^15 slots of
    N = 2^16; conv 32 -> 32 (288 rotations as one hoisted group, 288
    plaintext products), quadratic activation, conv, sum pooling, dense to 10
    classes, on a plain 4-level chain (60-bit q_0, 40-bit primes).  Images
    run one at a time; every image's logits are checked against the float64
    forward.  Prints its own JSON line."""
    import torch
    from oracle.forward import forward_chw
    from paper_2509_22857_amd.chw import ChwNetwork
    from paper_2509_22857_amd.ckks import Context
    from workloads import gen
    from workloads.nets import chw_spec
    from workloads.params import chw_chain
    ps = chw_chain(16, 4)
    spec = chw_spec(0, C=32, H=32, W=32, classes=10)
    ctx = Context.from_params(ps)
    delta = 2.0 ** ps.delta_log2
    net = ChwNetwork(ctx, spec, delta)
    t0 = time.time()
    keys = ctx.keygen(12345, net.steps)
    torch.cuda.synchronize()
    log(f"chw: {len(net.steps)} rotation keys, {keys.evk_bytes() / 2**30:.1f} GiB, {time.time() - t0:.1f}s")
    B = args.batch
    imgs = gen.images(777, B, *spec["image"])
    cts = [net.encrypt_image(keys, imgs[i], (1 << 20) + i) for i in range(B)]
    for i in range(min(args.warmup, B)):
        net.run(keys, cts[i])
    torch.cuda.synchronize()
    t0 = time.time()
    outs = [net.run(keys, c)["logits"] for c in cts]
    torch.cuda.synchronize()
    dt = time.time() - t0
    err = max(float(np.max(np.abs(net.decrypt_logits(keys, o) - forward_chw(spec, imgs[i])))) for i, o in enumerate(outs))
    log(f"chw: {B} images in {dt:.2f}s, logits within {err:.2e} of FP64")
    print(json.dumps({
        "metric": "encrypted images/s (CHW layout network, N=2^16, one image per ciphertext)",
        "value": round(B / dt, 4), "unit": "images/s", "n_gpus": 1, "steps": B, "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / B, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "chw_N65536", "channels": 32, "image": [32, 32], "classes": 10,
                   "levels": len(ps.q) - 1, "rotations_per_conv": sum(1 for t in net.rotation_steps(spec["image"][0]) if t),
                   "rotation_keys": len(net.steps), "key_GiB": round(keys.evk_bytes() / 2**30, 2)},
        "accuracy": {"max_abs_logit_err": err}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--images-per-pass", type=int, default=16,
                    help="images evaluated layer by layer together (bounds live ciphertexts)")
    ap.add_argument("--plain", type=int, default=2, help="images timed one at a time")
    ap.add_argument("--check", type=int, default=-1,
                    help="images whose logits are checked against FP64 (default: every image of the step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-out", default=os.path.join(ROOT, "tuning_fresh.json"),
                    help="where --tune fresh writes the choices it measured")
    ap.add_argument("--tune", default="cached", choices=["cached", "fresh", "off"],
                    help="autotuner: stored choices for this workload if any (else tune), re-tune, or defaults")
    ap.add_argument("--workload", default="resnet20", choices=["resnet20", "vgg", "micro", "serving", "chw"])
    ap.add_argument("--layout", default="slice", choices=["slice", "taps"],
                    help="slice-shared codebook (default) or one plaintext per tap")
    ap.add_argument("--pack", type=int, default=1,
                    help="images per ciphertext (slot packing, a separate labelled row; resnet20 only)")
    ap.add_argument("--clients", type=int, default=8, help="serving: clients with their own keys")
    ap.add_argument("--serve-rates", default="0.2,0.5,2,10",
                    help="serving: Poisson arrival rates (req/s), below and above capacity")
    ap.add_argument("--serve-requests", type=int, default=32, help="serving: requests per rate")
    ap.add_argument("--serve-max-images", type=int, default=8, help="serving: images per batch")
    ap.add_argument("--serve-streams", type=int, default=3, help="serving: concurrent batches")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the evaluator runs on a single MI355X "
              "(sharding across GPUs is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "micro":
        import torch
        from paper_2509_22857_amd import microbench
        calibration_copy(torch)
        print(json.dumps(microbench.run(batch=args.batch, reps=max(args.steps, 1), log=log)))
        return
    if args.workload == "serving":
        from paper_2509_22857_amd import serve_bench
        from oracle.forward import forward
        print(json.dumps(serve_bench.run(args, log, reference=forward)))
        return

    if args.pack > 1:
        run_packed(args)
        return
    if args.workload == "chw":
        run_chw(args)
        return

    import torch
    from paper_2509_22857_amd import ckks
    from paper_2509_22857_amd.ckks import Context
    from paper_2509_22857_amd.network import GpuNetwork
    from workloads import gen

    t0 = time.time()
    ps, spec = build_workload(args)
    log(f"spec built in {time.time() - t0:.1f}s; params {ps.name}: N=2^{ps.logN}, {len(ps.q)} Q + {len(ps.p)} P primes")
    ctx = Context.from_params(ps)
    delta = 2.0 ** ps.delta_log2
    t0 = time.time()
    net = GpuNetwork(ctx, spec, delta, delta, delta)
    torch.cuda.synchronize()
    log(f"layers on device in {time.time() - t0:.1f}s ({net.device_bytes() / 2**30:.1f} GiB plaintext codebooks)")
    t0 = time.time()
    keys = ctx.keygen(12345, net.steps)
    log(f"keys: {len(net.steps)} rotations + relin, {keys.evk_bytes() / 2**30:.1f} GiB, {time.time() - t0:.1f}s")
    B = args.batch
    imgs = gen.images(777, B, *spec["image"])
    t0 = time.time()
    cts = net.encrypt_images(keys, imgs, stream_base=1 << 20)
    torch.cuda.synchronize()
    log(f"encrypted {B} images in {time.time() - t0:.1f}s")

    stream = torch.cuda.current_stream()
    calibration_copy(torch)
    tuned = None
    if args.tune != "off":
        from paper_2509_22857_amd.autotune import tune_network, TUNING_FILE
        t0 = time.time()
        sample = cts[: min(B, args.images_per_pass)]
        key = f"{'vgg_N65536' if args.workload == 'vgg' else 'resnet20_ensemble_N65536'}/{len(sample)}"
        if args.tune == "fresh":
            # a fresh search writes its own cache file (--tune-out), never the committed choices
            os.makedirs(os.path.dirname(os.path.abspath(args.tune_out)), exist_ok=True)
            tuned = tune_network(net, keys, sample, cache=args.tune_out, key=key, log=log, refresh=True)
        else:
            tuned = tune_network(net, keys, sample, cache=TUNING_FILE, key=key, log=log, write=False)
        log(f"autotune ({args.tune}) in {time.time() - t0:.1f}s: { {k: v for k, v in tuned.items() if k != 'timings'} }")
        # per-layer key-switching form: measured (fresh) or the stored marks
        # for this workload and layout; the marks are part of the network
        # description, so a change rebuilds the layers (the keys stay valid:
        # both forms rotate by the same steps)
        from paper_2509_22857_amd.autotune import tune_hoisting
        from workloads.nets import set_hoisting
        hkey = f"{key}/{args.layout}/hoisting"
        marks = None
        if args.tune == "fresh":
            t0 = time.time()
            marks = tune_hoisting(net, keys, len(sample), log=log)
            data = json.load(open(args.tune_out)) if os.path.exists(args.tune_out) else {}
            data[hkey] = marks
            with open(args.tune_out, "w") as f:
                json.dump(data, f, indent=1)
            log(f"hoisting tuned in {time.time() - t0:.1f}s: {marks}")
        elif os.path.exists(TUNING_FILE):
            marks = json.load(open(TUNING_FILE)).get(hkey)
        current = [ly.get("hoist", "double") for ly in spec["layers"] if ly["op"] == "conv"]
        if marks and marks != current:
            del net
            torch.cuda.empty_cache()
            set_hoisting(spec, marks)
            net = GpuNetwork(ctx, spec, delta, delta, delta)
            torch.cuda.synchronize()
            log(f"layers rebuilt with the tuned hoisting marks {marks}")
        tuned["hoisting"] = marks or current
    for w in range(args.warmup):
        t0 = time.time()
        out, _ = net.run(keys, cts, images_per_pass=args.images_per_pass)
        torch.cuda.synchronize()
        log(f"warmup {w}: {time.time() - t0:.2f}s")

    ckks.prof_enable(True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.time()
    ev0.record(stream)
    for k in range(args.steps):
        out, _ = net.run(keys, cts, images_per_pass=args.images_per_pass)
        log(f"step {k} enqueued")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t_wall
    ms = ev0.elapsed_time(ev1)
    prof = {k: ckks.prof_query(k) for k in ckks.PROF_KERNELS}
    ckks.prof_enable(False)
    sec_per_step = ms / 1e3 / args.steps
    ips = B / sec_per_step
    log(f"batched: {sec_per_step:.2f}s per step of {B} images -> {ips:.3f} images/s (wall {wall:.1f}s)")

    # plain: one image at a time through the same kernels
    t_plain = 0.0
    nplain = min(args.plain, B)
    for i in range(nplain):
        torch.cuda.synchronize()
        a = time.time()
        net.run(keys, [cts[i]])
        torch.cuda.synchronize()
        t_plain += time.time() - a
    plain_ips = nplain / t_plain if nplain else None
    if plain_ips:
        log(f"plain: {plain_ips:.3f} images/s")
    # plain, as a captured HIP graph replayed per image
    graph_ips = None
    if nplain:
        from paper_2509_22857_amd.graph import GraphedPass
        gp = GraphedPass(net, keys, 1)
        torch.cuda.synchronize()
        a = time.time()
        for i in range(nplain):
            gp.run([cts[i]])
        torch.cuda.synchronize()
        graph_ips = nplain / (time.time() - a)
        log(f"plain, graph replay: {graph_ips:.3f} images/s")
        del gp

    # accuracy of the timed outputs against the FP64 forward
    from oracle.forward import forward
    max_err, agree = 0.0, 0
    nchk = B if args.check < 0 else min(args.check, B)
    for i in range(nchk):
        got = net.decrypt_logits(keys, out[i])
        ref = forward(spec, imgs[i])
        max_err = max(max_err, float(np.max(np.abs(got - ref))))
        agree += int(got.mean(0).argmax() == ref.mean(0).argmax())
    log(f"logits vs FP64: max abs err {max_err:.2e}, top-1 agree {agree}/{nchk}")

    # roofline of the dominant kernel class: HBM-bound classes against the
    # HBM peak, multiply-bound classes against the chip's 64-bit modular
    # multiply rate (4 full-rate 32x32->64 multiply-adds per 64-bit product,
    # 256 CUs x 64 lanes x 2.4 GHz / 4)
    tot = {k: v["ms"] for k, v in prof.items()}
    dom = max(tot, key=tot.get)
    kip = prof["kip"]
    kip_gbs = kip["bytes"] / (kip["ms"] / 1e3) / 1e9 if kip["ms"] > 0 else 0.0
    ks_cls = ("ntt_fwd", "ntt_inv", "bconv", "kip", "moddown")
    ks_ms = sum(prof[k]["ms"] for k in ks_cls)
    ks_gbs = sum(prof[k]["bytes"] for k in ks_cls) / (ks_ms / 1e3) / 1e9 if ks_ms > 0 else 0.0
    d = prof[dom]
    launches = max(d["launches"], 1)
    if dom in MUL_BOUND:
        achieved = d["work"] / (d["ms"] / 1e3) / 1e12 if d["ms"] > 0 else 0.0
        roof = {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3), "peak": MODMUL_PEAK_T,
                "unit": "T mod-mul/s", "frac": round(achieved / MODMUL_PEAK_T, 4), "traffic": None}
    else:
        achieved = d["bytes"] / (d["ms"] / 1e3) / 1e9 if d["ms"] > 0 else 0.0
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
    roof.update({"avg_launch_ms": round(d["ms"] / launches, 4), "launches": d["launches"],
                 "hbm_GBs": round(d["bytes"] / (d["ms"] / 1e3) / 1e9, 1) if d["ms"] > 0 else 0.0,
                 "alg_bytes_per_launch": round(d["bytes"] / launches)})
    wkey = workload_key(args, tuned)
    tr = measured_traffic(dom, wkey)
    log(f"traffic key {dom} {kernel_source_hash(dom)} {wkey}: {tr}")
    if tr is not None:
        roof["traffic"] = round(tr["bytes_per_launch"])
        roof["traffic_unit"] = "bytes/launch"
        roof["traffic_source"] = (f"replayed from profiles/{dom}_traffic.md: FETCH_SIZE and WRITE_SIZE counters of "
                                  "an earlier run of the same kernel sources and launch choices on this workload, "
                                  "not measured in this run")
    shares = {k: round(v / max(sum(tot.values()), 1e-9), 3) for k, v in tot.items()}
    busy = sum(tot.values()) / max(ms, 1e-9)
    log(f"profiled kernel time {sum(tot.values()) / 1e3:.2f}s of {ms / 1e3:.2f}s timed ({100 * busy:.1f}%)")
    rates = {k: {"GBs": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1),
                 "Tmul": round(v["work"] / (v["ms"] / 1e3) / 1e12, 3)} for k, v in prof.items() if v["ms"] > 0}
    log(f"kernel time shares: {shares}")
    log(f"kernel rates: {rates}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cw = prof["conv_contract"]["work"] + prof["dense_mac"]["work"]
        cpu = cpu_baseline(ps, spec, gpu_products_per_image=cw / (B * args.steps))
        log(f"cpu baseline: {cpu}")

    res = {
        "metric": ("encrypted images/s (VGG-style, N=2^16, batched)" if args.workload == "vgg" else
                   "encrypted images/s (ResNet-20-style ensemble, N=2^16, batched)"),
        "value": round(ips, 4),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": ("vgg_N65536" if args.workload == "vgg" else "resnet20_ensemble_N65536"),
                   "images_per_step": B,
                   "images_per_pass": min(B, args.images_per_pass), "members": spec["members"],
                   "layout": ("slice-shared columns, " if spec["layout"].get("slice_shared") else "per-tap masks, ")
                   + f"{spec['layout']['block']}-slot blocks",
                   "classes": spec["classes"], "k": spec["k"], "image": list(spec["image"]),
                   "levels": len(ps.q) - 1, "primes_q": len(ps.q), "primes_p": len(ps.p), "alpha": ps.alpha,
                   "tuned": ({k: v for k, v in tuned.items() if k != "timings"} if tuned else None)},
        "plain_images_per_s": round(plain_ips, 4) if plain_ips else None,
        "batched_over_plain": round(ips / plain_ips, 3) if plain_ips else None,
        "plain_graph_images_per_s": round(graph_ips, 4) if graph_ips else None,
        "key_switch_hbm": {"kernels": list(ks_cls), "achieved_GBs": round(ks_gbs, 1),
                           "frac": round(ks_gbs / HBM_PEAK_GBS, 4),
                           "kip_GBs": round(kip_gbs, 1), "kip_frac": round(kip_gbs / HBM_PEAK_GBS, 4)},
        "kernel_rates": rates,
        # whole-step HBM roofline fraction: the algorithmic bytes of every
        # profiled launch of the timed steps (inputs, keys and codebook tiles
        # counted once per launch that reads them) at 8 TB/s, over the
        # measured step time
        "throughput_hbm": {"alg_bytes_per_image": round(sum(v["bytes"] for v in prof.values()) / (B * args.steps)),
                           "frac": round(sum(v["bytes"] for v in prof.values()) / (HBM_PEAK_GBS * 1e9)
                                         / (ms / 1e3), 4)},
        "accuracy": {"max_abs_logit_err": max_err, "top1_agree": f"{agree}/{nchk}"},
        "kernel_time_share": shares,
        "profiled_kernel_busy": round(busy, 4),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
