"""Seeded random draws of the learned linewidth form.

The split of the candidate modes, the bootstrap counts and the initial
network weights are random inputs of the surrogate, drawn here once and
passed to both the oracle and the GPU path.  Nothing of the method's
arithmetic lives here.

* split: numpy default_rng(seed).permutation of the candidates; the first
  round(train_frac n) are the training rows, the next round(held_frac n)
  the held-out rows, the rest the rows the network may answer.
* member e (e = 0 .. M-1) draws from default_rng(seed + e): first the
  Glorot-uniform weights layer by layer (U(-l, l), l = sqrt(6 / (fan_in +
  fan_out)), zero biases), then n_train bootstrap indices in [0, n_train);
  counts[e] is their histogram.
* parameter layout: W0 [n_in][64], b0, W1..W3 [64][64] each followed by its
  bias, W4 [64][1], b4; row-major, concatenated.
"""
from __future__ import annotations

import dataclasses

import numpy as np

HIDDEN = 64
DEPTH = 4


@dataclasses.dataclass
class SurrogateDraws:
    perm: np.ndarray      # int64 [n]
    n_train: int
    n_held: int
    counts: np.ndarray    # float32 [M, n_train]
    params: np.ndarray    # float32 [M, P]
    params64: np.ndarray  # float64 [M, P], the same draws before rounding


def glorot_params(n_in, rng, hidden=HIDDEN, depth=DEPTH):
    sizes = [n_in] + [hidden] * depth + [1]
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=(a, b)).reshape(-1))
        parts.append(np.zeros(b))
    return np.concatenate(parts)


def surrogate_draws(n_candidates, n_in, members=5, seed=0, train_frac=0.1, held_frac=0.1):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n_candidates)
    n_train = max(1, int(round(train_frac * n_candidates)))
    n_held = max(1, int(round(held_frac * n_candidates)))
    if n_train + n_held > n_candidates:
        raise ValueError("too few candidate modes for the training and held-out splits")
    counts, params = [], []
    for e in range(members):
        r = np.random.default_rng(seed + e)
        params.append(glorot_params(n_in, r))
        idx = r.integers(0, n_train, size=n_train)
        counts.append(np.bincount(idx, minlength=n_train).astype(np.float64))
    p64 = np.stack(params)
    return SurrogateDraws(perm=perm, n_train=n_train, n_held=n_held,
                          counts=np.stack(counts).astype(np.float32),
                          params=p64.astype(np.float32), params64=p64)
