"""Batched evaluation of a whole encrypted network with graph replay.

One call evaluates the network for up to B independent ciphertexts (requests):
every layer is one set of batched launches (he_eval_dense_batch,
he_rescale_batch, he_square_batch), so keys and plaintext diagonals are read
once per batch instead of once per request.  All stage buffers are
preallocated; a HIP graph of the whole sequence, captured by the library
(he_graph_begin / he_graph_end) on a side stream, replays it with one launch
call.

Results are bit-identical to one-request-at-a-time evaluation: batching only
changes which launch a ciphertext rides in, never its arithmetic.
"""
from __future__ import annotations

from . import he
from .netplan import NetPlan


class NetworkRunner:
    def __init__(self, ctx: he.Context, plan: NetPlan, layers: list, batch: int):
        assert len(layers) == len(plan.layers)
        self.ctx, self.plan, self.layers, self.B = ctx, plan, layers, batch
        L = plan.L
        self.inputs = [ctx.new_ct(L, plan.scale) for _ in range(batch)]
        self.stages = []          # per layer: (dense_out, rescaled, squared, rescaled2)
        for li, lay in enumerate(plan.layers):
            lv = lay.level
            st = {"dense": [ctx.new_ct(lv) for _ in range(batch)],
                  "rs1": [ctx.new_ct(lv - 1) for _ in range(batch)]}
            if li + 1 < len(plan.layers):
                st["sq"] = [ctx.new_ct(lv - 1) for _ in range(batch)]
                st["rs2"] = [ctx.new_ct(lv - 2) for _ in range(batch)]
            self.stages.append(st)
        self.graphs = {}

    def outputs(self, b: int | None = None):
        return self.stages[-1]["rs1"][: (b or self.B)]

    def run(self, b: int | None = None, inputs=None):
        """Evaluate the first b slots (inputs default to self.inputs)."""
        b = b or self.B
        ctx = self.ctx
        cur = (inputs or self.inputs)[:b]
        for li, (d, st) in enumerate(zip(self.layers, self.stages)):
            cur = ctx.eval_dense_batch(cur, d, st["dense"][:b])
            cur = ctx.rescale_batch(cur, st["rs1"][:b])
            if "sq" in st:
                cur = ctx.square_batch(cur, st["sq"][:b])
                cur = ctx.rescale_batch(cur, st["rs2"][:b])
        return cur

    def capture(self, b: int | None = None):
        """Capture run(b) on self.inputs into a graph; returns a replay callable."""
        import torch
        b = b or self.B
        if b in self.graphs:
            return self.graphs[b]
        side = torch.cuda.Stream(device=self.ctx.device)
        side.wait_stream(torch.cuda.current_stream(self.ctx.device))
        with torch.cuda.stream(side):
            self.ctx.use_current_stream()
            self.run(b)                      # warm-up on the capture stream
            side.synchronize()
            g = self.ctx.capture(lambda: self.run(b))
        torch.cuda.current_stream(self.ctx.device).wait_stream(side)
        self.ctx.use_current_stream()
        self.graphs[b] = g
        return g
