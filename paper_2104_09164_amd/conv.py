"""Fast homomorphic convolution (paper, Methods, "Fast homomorphic
convolutions": merge-and-conquer) from the library's entry points.

A layer takes n_in punctured ciphertexts (valid entries at stride n_P) and
runs, on the device:
  (i)   pre: per group of n_P ciphertexts one linear transform (mask each by a
        plaintext, shift ciphertext p of the group right by p, sum) and a
        rescale: n_in / n_P merged ciphertexts;
  (ii)  the multi-channel convolution of the merged ciphertexts (one linear
        transform: kernel offsets n_P r_k as baby rotations, channel offsets as
        giant rotations);
  (iii) post: rotate-and-sum by n_P/2, ..., 1 and a rescale.
The plaintexts (masks, pre-rotated filter weights) come encoded from the model
owner, in coefficient form, as for he_linear_load.  For R requests per call
the context's workspace must be bound with max_batch >= R n_in and R n_out
and max_n2 >= max(n_P, channels per ciphertext).
"""
from __future__ import annotations


class FastConv:
    def __init__(self, ctx, level: int, nP: int, pre_giant, pre_pts, baby, giant, conv_pts, post, pt_scale: float):
        self.ctx, self.level, self.nP = ctx, level, nP
        self.pre = ctx.linear_load(level, [0], list(pre_giant), pre_pts, pt_scale)
        self.conv = ctx.linear_load(level - 1, list(baby), list(giant), conv_pts, pt_scale)
        self.post = list(post)
        self.merged = []

    def run(self, cts):
        """cts: R x n_in punctured inputs (request-major); returns R x n_out
        outputs.  Every step runs batched over the requests (plaintexts read
        once per batch)."""
        ctx, nP = self.ctx, self.nP
        n_in = self.conv.n_in * nP
        if len(cts) % n_in:
            raise ValueError(f"{len(cts)} inputs for layers of {n_in}")
        # groups of nP consecutive inputs are independent requests of the merge transform
        self.merged = ctx.rescale_batch(ctx.eval_linear_batch(list(cts), self.pre))
        z = ctx.eval_linear_batch(self.merged, self.conv)
        for t in self.post:
            rz = ctx.rotate_hoisted_batch(z, [t])
            z = [ctx.add(a, b) for a, b in zip(z, rz)]
        return ctx.rescale_batch(z)
