"""Serving measurement: a mix of encrypted ResNet-18-style and ResNet-20-style
requests from several clients arriving as a Poisson process.

  * ResNet-18-style: 64x64x3 inputs, stages 64/128/256/512 x 2 basic blocks,
    200 classes, one member, slot blocks of 8192 (64 rows of 64 under 64
    spare rows), its own tower chain of 18 levels.
  * ResNet-20-style: the headline ensemble (32x32x3, 16/32/64 x 3 blocks,
    100 classes, 4 members, blocks of 2048), tower chain of 20 levels.

Both run at N = 2^16 with 64 centroids per kernel column in the slice-shared
layout.  Every client owns its evaluation keys (resident for the whole run).
The one-at-a-time rate is measured first: requests of both networks run one
after another, each alone on the GPU.  Then, for each arrival rate, the same
number of requests (half per network, clients drawn at random) is replayed
in real time through the serving loop, which reports p50 / p99 latency
(arrival to logits ready), images/s, batches (and how many merged several
clients) and memory waits.
Synthetic data: seeded random weights of these shapes and uniform [0, 1]
images stand in for the datasets.
"""
from __future__ import annotations

import time

import numpy as np


def build(log, r18_calib: int = 4):
    import torch
    from . import ckks
    from .network import GpuNetwork, choose_hoisting
    from workloads import nets
    from workloads.params import resnet20_tower
    t0 = time.time()
    specs = {
        "resnet18": nets.resnet_spec(seed=5, members=1, widths=(64, 128, 256, 512), blocks=2, classes=200,
                                     image=(3, 64, 64), k=64, calib=r18_calib, block_slots=8192),
        "resnet20": nets.resnet_spec(seed=0, members=4, widths=(16, 32, 64), blocks=3, classes=100,
                                     image=(3, 32, 32), k=64, calib=8, block_slots=2048),
    }
    for spec in specs.values():
        spec["layout"]["slice_shared"] = True
    log(f"specs built in {time.time() - t0:.1f}s")
    chains = {"resnet18": resnet20_tower(levels=18), "resnet20": resnet20_tower(levels=20)}
    nets_on_gpu = {}
    for name, spec in specs.items():
        ps = chains[name]
        ctx = ckks.Context.from_params(ps)
        d = 2.0 ** ps.delta_log2
        # per-layer key-switching form (ResNet-18's wide low-level layers single-hoisted)
        nets.set_hoisting(spec, choose_hoisting(spec, ps.q, len(ps.p), d, d, d))
        log(f"{name}: hoisting {[ly.get('hoist', 'double') for ly in spec['layers'] if ly['op'] == 'conv']}")
        t0 = time.time()
        nets_on_gpu[name] = GpuNetwork(ctx, spec, d, d, d)
        torch.cuda.synchronize()
        log(f"{name}: {len(ps.q) - 1} levels, layers {nets_on_gpu[name].device_bytes() / 2**30:.1f} GiB "
            f"in {time.time() - t0:.1f}s")
    return specs, nets_on_gpu


def run(args, log, reference=None) -> dict:
    """reference: optional callable (spec, image) -> FP64 logits [M][K],
    supplied by the caller (the benchmark passes the oracle's forward); this
    package does not import the checker itself."""
    import torch
    from .serving import Request, Server, poisson_arrivals
    from workloads import gen
    specs, networks = build(log)
    clients = {f"c{i}": ("resnet18" if i % 2 == 0 else "resnet20") for i in range(args.clients)}
    keys = {}
    t0 = time.time()
    for i, (c, net) in enumerate(sorted(clients.items())):
        keys[(c, net)] = networks[net].ctx.keygen(7000 + i, networks[net].steps)
    torch.cuda.synchronize()
    kb = sum(k.evk_bytes() for k in keys.values())
    log(f"{len(keys)} clients' keys: {kb / 2**30:.1f} GiB in {time.time() - t0:.1f}s")
    free, total = torch.cuda.mem_get_info()
    budget = int(0.8 * free) + kb  # reset per rate once its requests are encrypted
    srv = Server(networks, budget, max_images=args.serve_max_images, n_streams=args.serve_streams)
    for (c, net), k in keys.items():
        srv.register_client(c, net, k)
    ws = {n: networks[n].working_set_bytes(1) / 2**30 for n in networks}
    log(f"budget {budget / 2**30:.1f} GiB (keys included); one-image working sets {ws}")

    # one at a time: `n_alone` requests of each network, each alone on the
    # GPU, one after another (single-request latency, and the rate of the
    # same 50/50 mix without serving)
    names = sorted(clients)
    alone, n_alone = {}, 2
    for net in ("resnet20", "resnet18"):
        pool = [x for x in names if clients[x] == net]
        ts = []
        for j in range(n_alone):
            c = pool[j % len(pool)]
            img = gen.images(99 + j, 1, *specs[net]["image"])
            cts = networks[net].encrypt_images(keys[(c, net)], img, stream_base=(1 << 30) + (j << 12))
            torch.cuda.synchronize()
            a = time.time()
            out, _ = networks[net].run(keys[(c, net)], cts)
            torch.cuda.synchronize()
            ts.append(time.time() - a)
            if j == 0 and reference is not None:
                got = networks[net].decrypt_logits(keys[(c, net)], out[0])
                err = float(np.max(np.abs(got - reference(specs[net], img[0]))))
                log(f"{net} alone {ts[-1]:.2f}s, logits vs FP64 max abs err {err:.2e}")
        alone[net] = float(np.mean(ts[1:] if len(ts) > 1 else ts))  # the first run warms up
    one_at_a_time = 2.0 / (alone["resnet18"] + alone["resnet20"])
    log(f"single request latency alone: {alone}; one at a time, 50/50 mix: {one_at_a_time:.3f} images/s")

    results = []
    rates = [float(r) for r in args.serve_rates.split(",")]
    for ri, rate in enumerate(rates):
        g = np.random.default_rng(100 + ri)
        arr = poisson_arrivals(rate, args.serve_requests, 200 + ri)
        reqs = []
        for i in range(args.serve_requests):
            net = "resnet18" if i % 2 == 0 else "resnet20"
            pool = [c for c in names if clients[c] == net]
            c = pool[int(g.integers(len(pool)))]
            img = gen.images(10_000 * (ri + 1) + i, 1, *specs[net]["image"])
            cts = networks[net].encrypt_images(keys[(c, net)], img, stream_base=((ri + 1) << 24) + (i << 12))
            reqs.append(Request(i, c, net, cts, float(arr[i])))
        torch.cuda.synchronize()
        last = [0]

        def progress(t, done, total):
            # a line about every eighth of the requests
            if done == total or done * 8 // total != last[0] * 8 // total:
                log(f"rate {rate} req/s: {done}/{total} served at {t:.0f} s")
            last[0] = done

        # the rate's encrypted requests sit in HBM outside the budget: admit
        # within 0.8 of what is free now, plus the resident keys
        free_now, _ = torch.cuda.mem_get_info()
        srv.budget = int(0.8 * free_now) + kb
        stats = srv.serve(reqs, progress=progress)
        torch.cuda.synchronize()
        per_net = {}
        for net in ("resnet18", "resnet20"):
            lat = np.array([r.done - r.arrival for r in reqs if r.net == net and r.done == r.done])
            if lat.size:
                per_net[net] = {"p50_s": round(float(np.percentile(lat, 50)), 3),
                                "p99_s": round(float(np.percentile(lat, 99)), 3)}
        stats = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in stats.items()}
        stats.update({"rate_req_s": rate, "per_network": per_net, "budget_GiB": round(srv.budget / 2**30, 1)})
        log(f"rate {rate:5.1f} req/s: {stats}")
        results.append(stats)
        # the next rate starts from the same free memory: the request
        # tensors go back to the device, not to torch's cache
        del reqs
        torch.cuda.empty_cache()
    cap = max(r["images_per_s"] for r in results if r["images_per_s"] == r["images_per_s"])
    return {
        "metric": "serving p50/p99 latency and images/s (ResNet-18/20-style mix, N=2^16, Poisson arrivals)",
        "unit": "s / images/s",
        "n_gpus": 1,
        "data": "synthetic",
        "dtype": "u64",
        "config": {"workload": "serving_mix_resnet18_resnet20_N65536", "clients": args.clients,
                   "requests_per_rate": args.serve_requests, "max_images_per_batch": args.serve_max_images,
                   "streams": args.serve_streams, "budget_GiB": round(budget / 2**30, 1)},
        "alone_s": {k: round(v, 3) for k, v in alone.items()},
        "one_at_a_time_images_per_s": round(one_at_a_time, 4),
        "rates": results,
        "capacity_images_per_s": cap,
        "served_over_one_at_a_time": round(cap / one_at_a_time, 3),
    }
