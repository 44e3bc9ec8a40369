"""Serving loop: continuous batching of encrypted inference requests.

A request is one client's encrypted image(s) for one of the served networks.
The server holds every network's layers and every registered client's
evaluation keys on the device, and runs a single host loop that

  * admits queued requests in arrival order while the HBM budget covers the
    working set of the batch they would start (keys are already resident),
    and sizes the scratch arena of the batch's stream for its largest call;
  * merges queued requests of the same network into one batch, whichever
    clients sent them: a key group gives every image its client's key set,
    so one client's images share its key-switching launches and all of them
    share every other launch (the contraction over the network's codebook,
    ModDown, rescale);
  * runs every admitted batch on its own HIP stream, one layer per step, with
    at most `window` layers enqueued ahead of the GPU, so batches admitted
    while others are on the device overlap with them;
  * retires a batch when its last layer's event has completed (or, when a
    library call of the batch failed, once its enqueued work has drained,
    marking its requests failed with the error) and releases its memory
    reservation, which lets the next queued requests in.  A stream keeps its
    scratch arena for its next batch (freeing device memory synchronises the
    whole device and would stall the batches still running); the arenas count
    against the budget and are freed only when an admission does not fit
    otherwise.

Each image's result does not depend on which other requests shared its batch
or ran beside it (every kernel computes each ciphertext independently, and a
key-switching launch only ever holds ciphertexts of one key set), so a
request gives the same ciphertexts alone and in the mix.  Latency is measured
from arrival to the moment the host sees the batch's last event complete.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import ckks


@dataclass
class Request:
    rid: int
    client: str
    net: str
    inputs: list            # [n_img][C] ciphertexts (resident)
    arrival: float          # seconds on the loop clock
    admitted: float | None = None
    done: float | None = None
    outputs: list | None = None
    batch_id: int | None = None
    error: str | None = None   # set when the request's batch failed


@dataclass
class _Batch:
    bid: int
    net: str
    client: str
    reqs: list
    stream: object
    gen: object
    reserve: int
    keys: object = None     # the batch's key set or key group
    events: collections.deque = field(default_factory=collections.deque)
    finished: bool = False
    result: object = None
    error: str | None = None


class Server:
    """networks: name -> GpuNetwork; clients are registered with their keys."""

    def __init__(self, networks: dict, budget_bytes: int, max_images: int = 16, n_streams: int = 4,
                 window: int = 2):
        import torch
        self.torch = torch
        self.networks = networks
        self.budget = int(budget_bytes)
        self.max_images = max_images
        self.window = window
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.arena = {st: 0 for st in self.streams}  # scratch arena bytes each stream holds
        self.keys = {}          # (client, net) -> KeyPair
        self.reserved = 0
        self.key_bytes = 0
        self.stats = collections.Counter()

    def register_client(self, client: str, net: str, keys: ckks.KeyPair):
        nbytes = keys.evk_bytes()
        if self.key_bytes + nbytes > self.budget:
            raise MemoryError(f"keys of client {client} do not fit the HBM budget")
        self.keys[(client, net)] = keys
        self.key_bytes += nbytes

    # ------------------------------------------------------------------ loop
    def serve(self, requests: list, clock=time.perf_counter, progress=None) -> dict:
        """Replay `requests` (sorted by arrival, seconds from the start) in
        real time and return per-request timing plus aggregate statistics.
        progress(t, done, total), if given, is called at every retirement."""
        torch = self.torch
        self.stats = collections.Counter()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        running: list[_Batch] = []
        free_streams = list(self.streams)
        t0 = clock()
        next_bid = 0
        max_running = 0
        n_done = 0
        waiting = None
        blocked = False  # a scratch reservation failed: admit again after a retirement
        while pending or queue or running:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            # ---- admission: FIFO head, merged with later requests of the same network
            while queue and free_streams and not blocked:
                head = queue[0]
                net = self.networks[head.net]
                room = self.budget - self.key_bytes
                if net.working_set_bytes(len(head.inputs)) > room:
                    # can never run: reject the head request
                    queue.popleft()
                    head.done = float("nan")
                    self.stats["rejected"] += 1
                    continue
                # the head plus later requests of the same network (any
                # client), as many as the image limit and the budget allow
                group, n_img = [], 0
                for r in list(queue):
                    if r.net == head.net and n_img + len(r.inputs) <= self.max_images \
                            and net.working_set_bytes(n_img + len(r.inputs)) <= room:
                        group.append(r)
                        n_img += len(r.inputs)
                stream = free_streams[-1]
                scratch = net.scratch_bytes(n_img)
                held = net.working_set_bytes(n_img) - scratch  # the batch's ciphertexts
                grow = max(0, scratch - self.arena[stream])

                def fits():
                    return self.reserved + sum(self.arena.values()) + held + grow <= room
                if not fits():
                    # idle streams' arenas go first
                    for st in free_streams:
                        if st is not stream and self.arena[st] > 0:
                            ckks.stream_release(st)
                            self.arena[st] = 0
                            self.stats["arena_releases"] += 1
                    if not fits():
                        if waiting != head.rid:
                            self.stats["waits_for_memory"] += 1  # requests that had to wait
                            waiting = head.rid
                        break
                # the batch's largest scratch is allocated now, so its calls
                # allocate nothing while it runs.  The budget counts bytes, not
                # contiguous blocks: when the device cannot hand out the block
                # after all, the group stays queued and admission resumes
                # after the next retirement (or, with nothing running, after
                # the cached blocks are returned)
                if grow > 0:
                    try:
                        ckks.stream_reserve(scratch, stream)
                        self.arena[stream] = scratch
                    except ckks.CkcError as err:
                        if "CKC_ENOMEM" not in str(err):
                            raise
                        self.stats["reserve_retries"] += 1
                        ckks.stream_release(stream)
                        self.arena[stream] = 0
                        torch.cuda.empty_cache()
                        if running:
                            blocked = True
                            break
                        if self.stats["reserve_retries_idle"] >= 1:
                            # nothing else holds memory and it still does not fit
                            queue.popleft()
                            head.done = float("nan")
                            head.error = str(err)
                            self.stats["rejected"] += 1
                            self.stats["reserve_retries_idle"] = 0
                            continue
                        self.stats["reserve_retries_idle"] += 1
                        continue
                self.stats["reserve_retries_idle"] = 0
                free_streams.pop()
                for r in group:
                    queue.remove(r)
                    r.admitted = now
                    r.batch_id = next_bid
                # inputs were written on the submitting stream
                stream.wait_stream(torch.cuda.current_stream())
                inputs = [row for r in group for row in r.inputs]
                members = sorted({r.client for r in group})
                if len(members) == 1:
                    bkeys = self.keys[(members[0], head.net)]
                else:
                    bkeys = ckks.KeyGroup([self.keys[(c, head.net)] for c in members],
                                          [members.index(r.client) for r in group for _ in r.inputs])
                    self.stats["mixed_batches"] += 1
                b = _Batch(next_bid, head.net, ",".join(members), group, stream,
                           net.stages(bkeys, inputs, stream=stream), held, bkeys)
                next_bid += 1
                self.reserved += held
                running.append(b)
                max_running = max(max_running, len(running))
                progressed = True
            # ---- progress: keep up to `window` layers of every batch enqueued
            for b in running:
                while b.events and b.events[0].query():
                    b.events.popleft()
                while not b.finished and len(b.events) < self.window:
                    try:
                        next(b.gen)
                    except StopIteration as stop:
                        b.finished = True
                        b.result = stop.value
                    except ckks.CkcError as err:
                        # the batch cannot complete: its requests fail once
                        # its enqueued work has drained; the loop goes on
                        b.finished = True
                        b.error = str(err)
                    ev = torch.cuda.Event()
                    ev.record(b.stream)
                    b.events.append(ev)
                    progressed = True
            # ---- retire
            for b in list(running):
                if b.finished and all(e.query() for e in b.events):
                    t_done = clock() - t0
                    if b.error is not None:
                        for r in b.reqs:
                            r.error = b.error
                            r.done = float("nan")
                        self.stats["failed"] += len(b.reqs)
                    else:
                        outs = b.result[0]
                        i = 0
                        for r in b.reqs:
                            r.outputs = outs[i:i + len(r.inputs)]
                            i += len(r.inputs)
                            r.done = t_done
                    running.remove(b)
                    # the stream keeps its arena for its next batch
                    free_streams.append(b.stream)
                    self.reserved -= b.reserve
                    b.keys = None
                    blocked = False
                    progressed = True
                    if progress is not None:
                        n_done += len(b.reqs)
                        progress(t_done, n_done, len(requests))
            if not progressed:
                # nothing to enqueue: wait a little for the GPU or the next arrival
                wait = 5e-4
                if pending and not queue and not running:
                    wait = max(0.0, min(0.05, pending[0].arrival - (clock() - t0)))
                time.sleep(wait)
        # the run is over: the streams' arenas go back to the device
        for st in self.streams:
            if self.arena[st] > 0:
                ckks.stream_release(st)
                self.arena[st] = 0
        served = [r for r in requests if r.done is not None and not math.isnan(r.done)]
        lat = np.array([r.done - r.arrival for r in served]) if served else np.zeros(1)
        span = (max(r.done for r in served) - min(r.arrival for r in requests)) if served else float("nan")
        n_images = sum(len(r.inputs) for r in served)
        return {
            "requests": len(requests),
            "served": len(served),
            "rejected": int(self.stats["rejected"]),
            "failed": int(self.stats["failed"]),
            "waits_for_memory": int(self.stats["waits_for_memory"]),
            "mixed_client_batches": int(self.stats["mixed_batches"]),
            "arena_releases": int(self.stats["arena_releases"]),
            "reserve_retries": int(self.stats["reserve_retries"]),
            "batches": next_bid,
            "max_concurrent_batches": max_running,
            "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()),
            "images_per_s": n_images / span if span and span > 0 else float("nan"),
            "span_s": span,
        }


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of `rate` requests/s:
    cumulative sums of seeded exponential gaps."""
    g = np.random.default_rng(seed)
    return np.cumsum(g.exponential(1.0 / rate, n))
