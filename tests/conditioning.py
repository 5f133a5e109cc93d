"""How strongly the method's result depends on rounding of the colour split, measured with the
oracle alone.  Test infrastructure (used by CPU pins and by GPU parity tests).

The library stores the total populations and the colour state (c, v) of the last collision, so
its red and blue densities carry an absolute rounding error of the order of the unit roundoff
times the total density, even where one colour is a tiny tail; the oracle stores the two
colours separately and resolves such tails to full relative precision.  Both are correct
evaluations of the method.  Where the method is well conditioned the difference stays at the
rounding level.  Where a discontinuous decision sits in the tail (n = 0 below |grad rho^N| = eps,
reading R6) and its outcome is multiplied by an O(1) quantity, the difference is amplified:
under the surface-energy rule (rho^N = cos(theta) on the wall) the gradient on the first fluid
row is O(1) in pure phases, so the curvature there, and the CSF force, depend at O(sigma) on the
direction of n one row further in, where |grad rho^N| is a rounding-sized tail.

colour_split_noise() moves a rounding-sized amount between the two colours of every population
where both are present (pure phases stay exact, as in the library); the spread of the oracle's
own results under such noise is the part of the result rounding decides.
"""
from __future__ import annotations

import numpy as np


def colour_split_noise(pops: np.ndarray, rng, rel: float) -> np.ndarray:
    """(2, 9, ny, nx) populations with rel * (f_R + f_B) * N(0, 1) moved from blue to red in
    every population that holds both colours (clipped so that neither goes negative)."""
    r, b = pops[0], pops[1]
    tot = r + b
    both = (r > 0) & (b > 0)
    d = np.where(both, np.clip(rel * tot * rng.standard_normal(tot.shape), -r, b), 0.0)
    out = pops.copy()
    out[0] = r + d
    out[1] = b - d
    return out


def fraction_rounded_to_fp32(pops: np.ndarray) -> np.ndarray:
    """(2, 9, ny, nx) populations whose red fraction f_R / (f_R + f_B) is rounded to FP32 in every
    population that holds both colours (totals kept): colour tails below the FP32 resolution of the
    total vanish, as they do in FP32 arithmetic."""
    r, b = pops[0], pops[1]
    tot = r + b
    both = (r > 0) & (b > 0)
    frac = np.where(both, (r / np.where(both, tot, 1.0)).astype(np.float32).astype(np.float64), 0.0)
    out = pops.copy()
    out[0] = np.where(both, frac * tot, r)
    out[1] = np.where(both, tot - out[0], b)
    return out


def one_step_sensitivity(make_oracle, pops: np.ndarray, rel: float, seeds=(11, 12, 13)):
    """One oracle step from `pops`, and the largest change of each output population when the
    input's colour split is perturbed: at level `rel` (several seeds), and by rounding each red
    fraction to FP32.  Returns (ref, spread)."""
    o = make_oracle()
    o.set_pops(pops)
    ref = o.step(1).pops()
    spread = np.zeros_like(ref)
    variants = [colour_split_noise(pops, np.random.default_rng(seed), rel) for seed in seeds]
    variants.append(fraction_rounded_to_fp32(pops))
    for v in variants:
        o = make_oracle()
        o.set_pops(v)
        spread = np.maximum(spread, np.abs(o.step(1).pops() - ref))
    return ref, spread


def run_spread(make_oracle, steps: int, rel: float, seed: int = 5) -> float:
    """Largest difference, after `steps` steps, between the oracle and the oracle with colour-split
    noise of level `rel` injected after every step (the accumulated effect of per-step rounding)."""
    a, b = make_oracle(), make_oracle()
    rng = np.random.default_rng(seed)
    for _ in range(steps):
        a.step(1)
        b.step(1)
        b.set_pops(colour_split_noise(b.pops(), rng, rel))
    return float(np.abs(a.pops() - b.pops()).max())
