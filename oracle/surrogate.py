"""FP64 host pieces of the learned linewidth form, written plainly for tests.

The paper restricts the scattering calculation to the irreducible wedge of
the q-mesh and maps the results back onto the full grid (its overview of the
2.0 computational changes); it gives no surrogate.  The surrogate readings
fixed here are:

* irreducible wedge: q' ~ q when q' = R q on the mesh for a point operation R
  of the crystal (lattice operation that maps the basis onto itself, masses
  included, up to a translation); the representative is the smallest flat
  index of the star.  This oracle only knows the 48 signed permutations of
  Cartesian axes (cubic holohedry), which covers the cubic test lattices.
* star map: Gamma(q, s) = mean of Gamma(rep(q), s') over the frequency
  cluster (|d nu| < 1e-4 THz) of s at the representative.
* features of mode (q, s): nu [THz], |v| [A/ps], branch one-hot (3 N_b), the
  ascending |components| of the shortest Cartesian image q + G (G over
  {-1,0,1} combinations of the reciprocal vectors), |q + G|, ln(1 + D+),
  ln(1 + D-) with the joint densities of states of `oracle.jdos`.
* training domain: a row is inside when each of its (standardised)
  features lies within that column's [min, max] over the training rows.
* gate score: (w / Gamma_pred) * spread * sd, the first-order conductivity
  error the ensemble's disagreement implies, w = star size * c(omega)/k_B *
  |v|^2, Gamma_pred = exp(mean * sd + mu); +inf outside the domain.
* gate threshold: held-out rows taken in ascending score, whole groups of
  equal score at a time; a group is accepted while
  |sum_acc w (1/Gamma_pred - 1/Gamma_true)| <= tol * sum_all w / Gamma_true.
  tau is the next float32 above the last accepted score (0 when nothing is
  accepted); rows with score < tau use the network.

This is test infrastructure.
"""
from __future__ import annotations

import itertools

import numpy as np

from .constants import TWO_PI
from .kappa import heat_capacity_kb
from .phonons import DEG_TOL_THZ, mesh_points, reciprocal


def cubic_operations():
    """The 48 signed permutation matrices (Cartesian)."""
    ops = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3))
            for i, (p, s) in enumerate(zip(perm, signs)):
                R[i, p] = s
            ops.append(R)
    return ops


def crystal_operations(model, tol=1e-6):
    """Cartesian point operations (among the cubic ones) of the crystal."""
    A = np.asarray(model.lattice, float)      # rows a_i
    Ainv = np.linalg.inv(A)
    frac = np.asarray(model.frac, float)
    mass = np.asarray(model.mass, float)
    out = []
    for R in cubic_operations():
        # R a_i in lattice coordinates must be integral
        M = (A @ R.T) @ Ainv
        if np.max(np.abs(M - np.rint(M))) > tol:
            continue
        # fractional positions x -> x @ M (row convention) + t
        img = frac @ np.rint(M)
        found = False
        for j in range(len(frac)):
            if abs(mass[j] - mass[0]) > 1e-9:
                continue
            t = frac[j] - img[0]
            ok = True
            for a in range(len(frac)):
                d = frac - (img[a] + t)
                d -= np.rint(d)
                hit = np.where((np.max(np.abs(d), axis=1) < tol)
                               & (np.abs(mass - mass[a]) < 1e-9))[0]
                if hit.size != 1:
                    ok = False
                    break
            if ok:
                found = True
                break
        if found:
            out.append(R)
    return out


def ibz_map(model, mesh):
    """ir_of_q (N_q,) int: the smallest flat mesh index in the star of q."""
    N = np.asarray(mesh)
    pts = mesh_points(mesh)                   # (N_q, 3) integer mesh coordinates
    B = reciprocal(model.lattice)             # rows b_i
    Binv = np.linalg.inv(B)
    ops = crystal_operations(model)
    nq = len(pts)
    ir = np.arange(nq)
    for q in range(nq):
        qc = (pts[q] / N) @ B
        best = q
        for R in ops:
            k = (R @ qc) @ Binv * N           # mesh coordinates of R q
            kr = np.rint(k)
            if np.max(np.abs(k - kr)) > 1e-6:
                continue
            kr = kr.astype(int) % N
            idx = (kr[0] * N[1] + kr[1]) * N[2] + kr[2]
            best = min(best, idx)
        ir[q] = best
    return ir


def star_sizes(ir_of_q):
    """Number of mesh points represented by each representative (0 elsewhere)."""
    return np.bincount(ir_of_q, minlength=len(ir_of_q))


def star_map(ir_of_q, omega, gamma_ir):
    nq, nb3 = omega.shape
    out = np.zeros((nq, nb3))
    for q in range(nq):
        r = ir_of_q[q]
        nu = omega[r] / TWO_PI
        for s in range(nb3):
            lo = s
            while lo > 0 and nu[lo] - nu[lo - 1] < DEG_TOL_THZ:
                lo -= 1
            hi = s
            while hi < nb3 - 1 and nu[hi + 1] - nu[hi] < DEG_TOL_THZ:
                hi += 1
            out[q, s] = np.mean(gamma_ir[r, lo:hi + 1])
    return out


def features(model, mesh, omega, vel, dplus, dminus, modes):
    """Feature rows (n, 3 N_b + 8) of the listed flat mode indices."""
    N = np.asarray(mesh)
    pts = mesh_points(mesh)
    nq, nb3 = omega.shape
    B = reciprocal(model.lattice)
    rows = []
    for m in modes:
        q, s = divmod(int(m), nb3)
        f = [omega[q, s] / TWO_PI, np.linalg.norm(vel[q, s])]
        f += [1.0 if b == s else 0.0 for b in range(nb3)]
        best = None
        for G in itertools.product((-1, 0, 1), repeat=3):
            qc = (pts[q] / N + np.asarray(G)) @ B
            L = float(qc @ qc)
            if best is None or L < best[0] - 1e-12:
                best = (L, qc)
        f += sorted(np.abs(best[1]).tolist())
        f += [np.sqrt(best[0]), np.log1p(dplus[q, s]), np.log1p(dminus[q, s])]
        rows.append(f)
    return np.asarray(rows, float).reshape(len(modes), nb3 + 8)


def standardize(X, n_fit):
    """Columns standardised with the mean and population std of the first n_fit rows."""
    mu = X[:n_fit].mean(axis=0)
    sd = X[:n_fit].std(axis=0)
    sd = np.where(sd > 1e-10, sd, 1.0)
    return (X - mu) / sd, mu, sd


def domain_inside(X, n_fit):
    lo = X[:n_fit].min(axis=0)
    hi = X[:n_fit].max(axis=0)
    return np.all((X >= lo) & (X <= hi), axis=1)


def gate_score(mean, spread, y_mu_sd, weight, inside=None):
    mu, sd = float(y_mu_sd[0]), float(y_mu_sd[1])
    gp = np.exp(np.asarray(mean, float) * sd + mu)
    s = weight / gp * np.asarray(spread, float) * sd
    if inside is not None:
        s = np.where(inside, s, np.inf)
    return s


def mode_weights(omega_m, vel_m, T, star):
    """w = star size * c/k_B * |v|^2 of each row."""
    return star * heat_capacity_kb(omega_m, T) * np.sum(vel_m * vel_m, axis=-1)


def gate_threshold(gamma_true, gamma_pred, score, weight, tol):
    spread = np.asarray(score, np.float32)
    ref = np.sum(weight / gamma_true)
    diff = weight / gamma_pred - weight / gamma_true
    acc = 0.0
    tau = np.float32(0.0)
    for v in np.unique(spread):
        acc_new = acc + np.sum(diff[spread == v])
        if abs(acc_new) <= tol * abs(ref):
            acc = acc_new
            tau = np.nextafter(v, np.float32(np.inf))
        else:
            break
    return np.float32(tau)
