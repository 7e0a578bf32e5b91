"""Sequencing of the learned linewidth form over the library's entry points.

Every numerical step runs in libkaldo (HIP kernels, or host C++ for the
irreducible wedge); this module only orders the calls, lays out the mode
lists and moves the random draws, which the caller passes in.

Order of work (all on the caller's current stream):
  1. irreducible wedge of the mesh (host), star sizes;
  2. candidate rows = physical modes (nu >= nu_min) of the representatives,
     permuted by the draws into [training | held-out | rest];
  3. exact linewidths of the training and held-out rows;
  4. joint density of states of every candidate row, features, standardised
     with the training rows' statistics; targets ln Gamma of the training rows;
  5. ensemble training, inference on every row;
  6. gate: rows outside the training rows' feature ranges, and rows whose
     score (first-order conductivity error implied by the ensemble's
     disagreement) reaches the threshold calibrated on the held-out rows,
     go to the exact path;
  7. exact linewidths of the fallback rows; network values for the others;
  8. star map onto the full mesh.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import kaldo as K

TWO_PI = 2.0 * np.pi


@dataclasses.dataclass
class LearnedResult:
    gamma: torch.Tensor       # [N_q, nb3] full mesh, rad/ps
    gamma_ir: torch.Tensor    # [N_q, nb3], filled at the representatives
    modes: torch.Tensor       # int32 candidate rows [training | held-out | rest]
    n_train: int
    n_held: int
    n_fallback: int
    tau: float
    mean: torch.Tensor        # standardised ln Gamma, ensemble mean per row
    spread: torch.Tensor      # ensemble std per row
    score: torch.Tensor       # gate score per row (+inf outside the training domain)
    inside: torch.Tensor      # 1 where the row lies in the training rows' feature ranges
    y_mu_sd: torch.Tensor
    losses: torch.Tensor | None


class Wedge:
    """Irreducible wedge of a mesh for one crystal (host arrays and device copies)."""

    def __init__(self, lattice, frac, mass, mesh):
        self.mesh = tuple(int(x) for x in mesh)
        self.ir_of_q, self.star_size, self.n_ops, self.n_ir = K.mesh_ibz(lattice, frac, mass, mesh)
        self.reps = np.flatnonzero(self.ir_of_q == np.arange(len(self.ir_of_q))).astype(np.int32)
        self.ir_dev = torch.from_numpy(self.ir_of_q).cuda()
        self.star_dev = torch.from_numpy(self.star_size).cuda()

    def rep_modes(self, nb3):
        return (self.reps[:, None] * nb3 + np.arange(nb3)[None, :]).reshape(-1).astype(np.int32)


def candidate_modes(wedge: Wedge, omega, nb3, nu_min_thz):
    """Physical modes of the representatives (flat indices, ascending)."""
    rm = wedge.rep_modes(nb3)
    nu = omega.reshape(-1)[torch.from_numpy(rm).cuda().long()].cpu().numpy() / TWO_PI
    return rm[nu >= nu_min_thz]


def plain_ibz_linewidths(c, wedge: Wedge, omega, evec, vel, T, broadening, precision=K.FP32):
    """Exact linewidths on every representative mode, star-mapped to the mesh."""
    nq = len(wedge.ir_of_q)
    g_ir = torch.zeros(nq, c.nb3, dtype=torch.float64, device="cuda")
    sub = torch.from_numpy(wedge.rep_modes(c.nb3)).cuda()
    K.linewidths(c, wedge.mesh, omega, evec, vel, T, broadening, precision, subset=sub, out=g_ir)
    return K.star_map(wedge.mesh, c.nb3, wedge.ir_dev, omega, g_ir)


def learned_linewidths(c, wedge: Wedge, omega, evec, vel, T, broadening, candidates, draws, *,
                       steps=200, lr=2e-2, tol=0.01, precision=K.FP32, keep_losses=False):
    """Linewidths on the full mesh from the learned form.

    candidates: flat mode indices the draws' permutation applies to (normally
    `candidate_modes`); draws: a `synthetic.draws.SurrogateDraws`-like object
    with perm, n_train, n_held, counts [M, n_train], params [M, P]."""
    nq = len(wedge.ir_of_q)
    nb3 = c.nb3
    mesh = wedge.mesh
    order = np.asarray(candidates, np.int32)[np.asarray(draws.perm)]
    n_tr, n_ho = int(draws.n_train), int(draws.n_held)
    n_known = n_tr + n_ho
    modes = torch.from_numpy(np.ascontiguousarray(order)).cuda()
    g_ir = torch.zeros(nq, nb3, dtype=torch.float64, device="cuda")
    K.linewidths(c, mesh, omega, evec, vel, T, broadening, precision, subset=modes[:n_known], out=g_ir)
    dp, dm = K.jdos(c, mesh, omega, vel, broadening, subset=modes)
    X = K.surrogate_features(c, mesh, omega, vel, dp, dm, modes)
    K.standardize(X, n_tr)
    y, y_mu_sd = K.surrogate_targets(g_ir, modes[:n_tr])
    params = torch.from_numpy(np.ascontiguousarray(draws.params, np.float32)).cuda()
    counts = torch.from_numpy(np.ascontiguousarray(draws.counts, np.float32)).cuda()
    losses, _ = K.mlp_train(X[:n_tr], y, counts, params, steps, lr, losses=keep_losses)
    mean, spread = K.mlp_predict(X, params)
    inside = K.surrogate_domain(X, n_tr)
    score = K.gate_score(modes, mean, spread, y_mu_sd, omega, vel, wedge.star_dev, nb3, T, inside)
    tau = K.gate_calibrate(modes[n_tr:n_known], g_ir, mean[n_tr:n_known], y_mu_sd,
                           score[n_tr:n_known], omega, vel, wedge.star_dev, nb3, T, tol)
    computed_h = np.zeros(nq * nb3, np.uint8)
    computed_h[order[:n_known]] = 1
    computed = torch.from_numpy(computed_h).cuda()
    fb, n_fb = K.gate_select(modes[n_known:], score[n_known:], tau, computed)
    n_fallback = int(n_fb.item())
    if n_fallback:
        K.linewidths(c, mesh, omega, evec, vel, T, broadening, precision, subset=fb[:n_fallback],
                     out=g_ir)
    K.surrogate_fill(modes[n_known:], mean[n_known:], y_mu_sd, computed, g_ir)
    gamma = K.star_map(mesh, nb3, wedge.ir_dev, omega, g_ir)
    return LearnedResult(gamma=gamma, gamma_ir=g_ir, modes=modes, n_train=n_tr, n_held=n_ho,
                         n_fallback=n_fallback, tau=float(tau.item()), mean=mean, spread=spread,
                         score=score, inside=inside,
                         y_mu_sd=y_mu_sd, losses=losses)
