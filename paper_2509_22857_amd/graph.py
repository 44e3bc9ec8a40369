"""Network passes captured as HIP graphs.

A pass over a fixed number of images enqueues the same kernels with the same
arguments every time; only the input ciphertexts change.  GraphedPass runs
the pass once eagerly on its own stream (which creates the lazily built
device tables and grows that stream's scratch arena to the pass's needs),
then captures a second pass into a HIP graph whose input and output
ciphertext buffers are static.  Every later pass copies the new inputs into
the static buffers and replays the graph: the layer schedule is launched by
one call instead of one host call per kernel.  The evaluation paths make no
synchronising or allocating HIP call once the arena is warm, and no memset
nodes, so the captured graph is the eager schedule.
"""
from __future__ import annotations


class GraphedPass:
    def __init__(self, net, keys, n_img: int, in_scale: float | None = None):
        import torch
        self.torch = torch
        self.net = net
        ctx = net.ctx
        C = net.spec["image"][0]
        L = len(ctx.q) - 1
        scale = float(in_scale if in_scale is not None else net.in_scale)
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.inputs = [[ctx.new_ct(L, 2, scale) for _ in range(C)] for _ in range(n_img)]
            for row in self.inputs:
                for ct in row:
                    ct.buf.zero_()
        self.stream.synchronize()
        # eager warm-up pass on the capture stream
        net.run(keys, self.inputs, stream=self.stream)
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self.outputs, _ = net.run(keys, self.inputs, stream=self.stream)
        self.stream.synchronize()

    def run(self, inputs):
        """inputs: [n_img][C] ciphertexts (same level and scale as captured).
        Returns the static output ciphertexts, overwritten by the next run."""
        for srow, irow in zip(self.inputs, inputs):
            for s, x in zip(srow, irow):
                if x.level != s.level or abs(x.scale / s.scale - 1.0) > 2.0 ** -30:
                    raise ValueError("input level or scale differs from the captured pass")
                s.buf.copy_(x.buf)
        self.graph.replay()
        return self.outputs
