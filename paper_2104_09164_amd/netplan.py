"""Host-side plan of an encrypted dense network (library side).

A network is dense layers y = W x + b with the square activation between
them (paper, Methods, "Non-convolutional layers": bias and polynomial
activation collapsed per feature).  Evaluation order with lazy rescaling
(Methods, "Algorithmic and cryptographic optimizations", lazy rescaling):
dense -> rescale -> square -> rescale -> ... -> dense -> rescale.

This module only does bookkeeping: levels, scales (IEEE doubles updated by
*Delta_w, by squaring and by /q_l, in that order), the rotation steps each
layer needs (baby steps 1..n1-1, giant steps n1*j, rotate-and-sum n/2..m),
and the per-inference operation counts.  A layer with qp set runs in the
lazy-ModDown form (diagonals over Q_l u P, one ModDown per inner sum instead of
one per baby step); like n1 it changes the rounding, so it is part of the plan.
So is rs_bits: the rotate-and-sum as hoisted groups of that many bits of the
shift index (0 = the sequential log2(n/m) key switches).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class LayerPlan:
    m: int
    n: int
    n1: int
    level: int            # level the layer is evaluated at
    in_scale: float
    pt_scale: float
    qp: bool = False      # lazy-ModDown form (HE_DENSE_QP)
    rs_bits: int = 0      # rotate-and-sum: 0 sequential, b > 0 hoisted groups of b bits (HE_DENSE_RS)

    @property
    def n2(self) -> int:
        return self.m // self.n1

    @property
    def bias_scale(self) -> float:
        return self.in_scale * self.pt_scale

    def rs_amounts(self) -> list[int]:
        """Rotation amounts of the rotate-and-sum (sequential n/2 .. m, or the
        k t of each hoisted group, most significant group first)."""
        if self.rs_bits <= 0:
            s, t = [], self.n // 2
            while t >= self.m:
                s.append(t)
                t //= 2
            return s
        left, s = (self.n // self.m).bit_length() - 1, []
        while left > 0:
            b = min(self.rs_bits, left)
            left -= b
            s += [k * (self.m << left) for k in range(1, 1 << b)]
        return s

    def rs_groups(self) -> int:
        """Key switches (sequential) or hoisted groups of the rotate-and-sum."""
        total = (self.n // self.m).bit_length() - 1
        return total if self.rs_bits <= 0 else -(-total // self.rs_bits)

    def steps(self) -> list[int]:
        return list(range(1, self.n1)) + [self.n1 * j for j in range(1, self.n2)] + self.rs_amounts()

    def rs_count(self) -> int:
        c, t = 0, self.n // 2
        while t >= self.m:
            c += 1
            t //= 2
        return c

    def moddowns(self) -> int:
        """ModDowns of one evaluation: one per baby step, or one per inner sum
        in the lazy form, plus one per giant step and rotate-and-sum step."""
        return ((self.n2 if self.qp else 0) if self.n1 > 1 else 0) + (0 if self.qp else self.n1 - 1) \
            + (self.n2 - 1) + self.rs_groups()


@dataclass
class NetPlan:
    log_n: int
    q: list[int]
    p: list[int]
    alpha: int
    scale: float
    layers: list[LayerPlan] = field(default_factory=list)
    out_level: int = 0
    out_scale: float = 0.0

    @property
    def slots(self) -> int:
        return 1 << (self.log_n - 1)

    @property
    def L(self) -> int:
        return len(self.q) - 1

    @property
    def dnum(self) -> int:
        return -(-len(self.q) // self.alpha)

    def steps(self) -> list[int]:
        s = set()
        for lay in self.layers:
            s.update(lay.steps())
        return sorted(s)

    def max_n1(self) -> int:
        return max(l.n1 for l in self.layers)

    def max_n2(self) -> int:
        return max(l.n2 for l in self.layers)

    def op_counts(self) -> dict:
        ks = sum((l.n1 - 1) + (l.n2 - 1) + len(l.rs_amounts()) for l in self.layers) + (len(self.layers) - 1)
        return {"key_switches": ks, "multplain": sum(l.m for l in self.layers),
                "rescales": 2 * len(self.layers) - 1, "squares": len(self.layers) - 1,
                "hoisted_modups": sum(1 for l in self.layers if l.n1 > 1),
                "moddowns": sum(l.moddowns() for l in self.layers) + (len(self.layers) - 1),
                "lazy_moddown_layers": [li for li, l in enumerate(self.layers) if l.qp],
                "hoisted_rotate_and_sum_bits": [l.rs_bits for l in self.layers]}


def plan_network(log_n: int, q, p, alpha: int, scale_bits: int, shapes) -> NetPlan:
    """shapes: [(m, n, n1[, qp[, rs_bits]]), ...] from the first layer to the last."""
    pl = NetPlan(log_n, list(q), list(p), alpha, float(2 ** scale_bits))
    level, s = pl.L, pl.scale
    for li, shp in enumerate(shapes):
        m, n, n1 = shp[:3]
        lay = LayerPlan(m, n, n1, level, s, pl.scale, bool(shp[3]) if len(shp) > 3 else False,
                        int(shp[4]) if len(shp) > 4 else 0)
        pl.layers.append(lay)
        s = s * lay.pt_scale
        s = s / pl.q[level]
        level -= 1
        if li + 1 < len(shapes):
            s = s * s
            s = s / pl.q[level]
            level -= 1
        if level < 0:
            raise ValueError("modulus chain too short for this network")
    pl.out_level, pl.out_scale = level, s
    return pl


# Bounds of the fold: the square's input is shifted by d = b / (2a) and the
# constant a d^2 = b^2 / (4a) is cancelled by the next bias.  Both grow as |a|
# shrinks: the encrypted values grow with |d| (eating scale headroom) and the
# encrypted a (h + d)^2 carries a rounding error proportional to a d^2 that the
# bias no longer cancels.  Within these bounds the folded networks stay inside
# the 2^-12 logit tolerance at the configured scales; beyond them the fold is
# refused.
FOLD_MAX_SHIFT = 8.0
FOLD_MAX_CANCEL = 8.0


def fold_quadratic_activations(weights, biases, acts):
    """Collapse per-feature quadratic activations a x^2 + b x + c (paper,
    "Non-convolutional layers": bias, batch normalisation and the polynomial
    activation become one polynomial per feature) into the adjacent dense
    layers, so that the encrypted network only squares:
        a x^2 + b x + c = a (x + d)^2 + e,   d = b / (2a),  e = c - a d^2,
    d moves into the bias of the layer before, a scales the columns of the
    next layer's weights and W_next e moves into its bias.  Needs a != 0 in
    every feature, |b / 2a| <= FOLD_MAX_SHIFT and |b^2 / 4a| <= FOLD_MAX_CANCEL
    (ValueError otherwise).  Returns new (weights, biases) lists (FP64); the network
    W_L(... (W_1 x + b_1)^2 ...) + b_L with them equals the original one."""
    Ws = [np.array(W, dtype=np.float64) for W in weights]
    bs = [np.array(b, dtype=np.float64) for b in biases]
    for i, (a, b, c) in enumerate(acts):
        a, b, c = (np.asarray(v, dtype=np.float64) for v in (a, b, c))
        if np.any(a == 0):
            raise ValueError("a quadratic activation with a = 0 cannot be folded into a square")
        d = b / (2.0 * a)
        if np.max(np.abs(d)) > FOLD_MAX_SHIFT or np.max(np.abs(a * d * d)) > FOLD_MAX_CANCEL:
            raise ValueError(f"activation {i}: a too small for its b (|b / 2a| up to {np.max(np.abs(d)):.3g}, "
                             f"|b^2 / 4a| up to {np.max(np.abs(a * d * d)):.3g}; the fold allows "
                             f"{FOLD_MAX_SHIFT} and {FOLD_MAX_CANCEL})")
        e = c - a * d * d
        bs[i] = bs[i] + d
        bs[i + 1] = bs[i + 1] + Ws[i + 1] @ e
        Ws[i + 1] = Ws[i + 1] * a[None, :]
    return Ws, bs


# Workload presets (ring, primes by bit size, digit size, scale, layer shapes).
PRESETS = {
    "cfg1": dict(log_n=13, q_bits=[45] + [35] * 3, p_bits=[45], alpha=1, scale_bits=35,
                 shapes=[(64, 256, 8), (2, 64, 2)], sigma=0.05),
    "cfg3": dict(log_n=15, q_bits=[60] + [40] * 6, p_bits=[60] * 2, alpha=2, scale_bits=40,
                 shapes=[(128, 1024, 32), (2, 128, 2)], sigma=0.03),
    "cfg4": dict(log_n=16, q_bits=[60] + [45] * 10, p_bits=[60] * 3, alpha=3, scale_bits=45,
                 shapes=[(256, 4096, 16), (64, 256, 8), (2, 64, 2)], sigma=0.02),
}


def tuned_shapes(name: str, tuned: dict | None, tuned_n1: bool = True) -> list:
    """Layer shapes of a preset with the autotuner's plan choices: its n1 and
    lazy-ModDown flags (tuned_n1), or the preset's n1 with the flags the
    tuner found best for it."""
    shapes = [tuple(s) for s in PRESETS[name]["shapes"]]
    if not tuned:
        return shapes
    rs = tuned.get("rs_bits") or [0] * len(shapes)
    if tuned_n1 and tuned.get("n1"):
        qp = tuned.get("qp") or [False] * len(shapes)
        return [(m, n, n1, bool(f), int(r)) for (m, n, _), n1, f, r in zip(shapes, tuned["n1"], qp, rs)]
    qp = tuned.get("qp_preset") or [False] * len(shapes)
    return [(m, n, n1, bool(f), int(r)) for (m, n, n1), f, r in zip(shapes, qp, rs)]


def preset_plan(name: str, shapes=None) -> NetPlan:
    from . import he
    c = PRESETS[name]
    q, p = he.prime_chain(c["log_n"], c["q_bits"], c["p_bits"])
    return plan_network(c["log_n"], q, p, c["alpha"], c["scale_bits"], shapes or c["shapes"])
