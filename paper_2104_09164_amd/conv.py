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
owner, in coefficient form, as for he_linear_load.
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
        ctx, nP = self.ctx, self.nP
        if len(cts) % nP:
            raise ValueError(f"{len(cts)} inputs for groups of {nP}")
        self.merged = [ctx.rescale(ctx.eval_linear(cts[a * nP:(a + 1) * nP], self.pre)[0])
                       for a in range(len(cts) // nP)]
        outs = ctx.eval_linear(self.merged, self.conv)
        res = []
        for z in outs:
            for t in self.post:
                z = ctx.add(z, ctx.rotate(z, t))
            res.append(ctx.rescale(z))
        return res
