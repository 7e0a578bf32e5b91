"""Pins of the oracle's JDOS and MLP (the learned-form inputs and network)."""
import numpy as np
import pytest

from oracle import jdos as ojdos
from oracle import mlp
from oracle import phonons
from oracle.constants import TWO_PI
from synthetic import configs, models

B_FIXED = configs.Broadening(adaptive=False)
B_ADAPT = configs.Broadening(adaptive=True)


def test_jdos_matches_momentum_enumeration():
    """Brute force: partners found by testing q + q1 + q2 in the reciprocal
    lattice over all (q1, q2), not by mesh index arithmetic."""
    m = models.random_cell(5, 2)
    mesh = (2, 2, 3)
    om, ev, ve = phonons.phonons(m, mesh)
    dp, dm = ojdos.jdos(m, mesh, om, ve, B_FIXED)
    pts = phonons.mesh_points(mesh) / np.asarray(mesh, float)
    nq, nb3 = om.shape
    sig = TWO_PI * 0.1
    nu = om / TWO_PI
    for q in range(nq):
        for s in range(nb3):
            if nu[q, s] < 0.1:
                assert dp[q, s] == 0.0 and dm[q, s] == 0.0
                continue
            bp = bm = 0.0
            for q1 in range(nq):
                for q2 in range(nq):
                    tot = pts[q] + pts[q1] + pts[q2]
                    if np.max(np.abs(tot - np.round(tot))) > 1e-9:
                        continue
                    for a in range(nb3):
                        for b in range(nb3):
                            if nu[q1, a] < 0.1 or nu[q2, b] < 0.1:
                                continue
                            xp = (om[q, s] + om[q1, a]) - om[q2, b]
                            xm = (om[q, s] - om[q1, a]) - om[q2, b]
                            if abs(xp) < 2 * sig:
                                bp += np.exp(-xp * xp / sig ** 2) / (np.sqrt(np.pi) * sig)
                            if abs(xm) < 2 * sig:
                                bm += np.exp(-xm * xm / sig ** 2) / (np.sqrt(np.pi) * sig)
            assert abs(dp[q, s] - bp / nq) <= 1e-12 * max(1.0, bp)
            assert abs(dm[q, s] - bm / nq) <= 1e-12 * max(1.0, bm)


def test_jdos_process_sum_rule():
    """With a fixed width, every coalescence a + b -> c is the decay c -> a + b
    of another mode: sum_mu D+ = sum_mu D- exactly (up to rounding)."""
    m = models.diamond()
    mesh = (4, 4, 4)
    om, ev, ve = phonons.phonons(m, mesh)
    dp, dm = ojdos.jdos(m, mesh, om, ve, B_FIXED)
    assert np.all(dp >= 0) and np.all(dm >= 0)
    assert abs(dp.sum() - dm.sum()) <= 1e-12 * dp.sum()
    assert dp.sum() > 0


def test_mlp_gradient_matches_complex_step():
    """Back-propagated gradient vs the complex-step derivative
    Im L(p + i h e_k) / h (exact to rounding: every op of the loss is
    analytic), and vs central differences."""
    rng = np.random.default_rng(0)
    X = rng.normal(size=(23, 7))
    y = rng.normal(size=23)
    c = rng.integers(0, 3, size=23).astype(float)
    c[0] = 1.0
    params = mlp.init_params(7, np.random.default_rng(1))
    for p in params[1::2]:
        p[:] = rng.normal(scale=0.1, size=p.shape)
    loss, grads = mlp.loss_and_grad(params, X, y, c)
    flat = mlp.flatten(params)
    gflat = mlp.flatten(grads)
    def loss_c(f):
        ps = mlp.unflatten(f, 7)
        yh, _ = mlp.forward(ps, X.astype(complex))
        r = yh - y
        return np.sum(c * r * r) / c.sum()

    h = 1e-30
    for k in rng.choice(flat.size, 80, replace=False):
        fc = flat.astype(complex)
        fc[k] += 1j * h
        cs = loss_c(fc).imag / h
        assert abs(cs - gflat[k]) <= 1e-10 * max(1e-3, abs(gflat[k]))
        fp, fm = flat.copy(), flat.copy()
        fp[k] += 1e-5
        fm[k] -= 1e-5
        fd = (mlp.loss_and_grad(mlp.unflatten(fp, 7), X, y, c)[0]
              - mlp.loss_and_grad(mlp.unflatten(fm, 7), X, y, c)[0]) / 2e-5
        assert abs(fd - gflat[k]) <= 1e-7 * max(1e-3, abs(gflat[k])) + 1e-11


def test_adam_first_step_moves_every_weight_by_lr():
    """First Adam step: m^ = g, v^ = g^2, so |dp| = lr |g| / (|g| + eps)."""
    rng = np.random.default_rng(3)
    X = rng.normal(size=(30, 5))
    y = np.sin(X @ rng.normal(size=5))
    params = mlp.init_params(5, np.random.default_rng(4))
    loss, g = mlp.loss_and_grad(params, X, y, np.ones(30))
    old = [p.copy() for p in params]
    new = mlp.Adam(params, lr=1e-3).step(params, g)
    for a, b, gg in zip(old, new, g):
        expect = 1e-3 * np.abs(gg) / (np.abs(gg) + 1e-8)
        assert np.allclose(np.abs(a - b), expect, rtol=1e-9, atol=1e-15)


def test_mlp_training_reduces_loss():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(120, 6))
    y = np.tanh(X @ rng.normal(size=6)) + 0.1 * X[:, 0] ** 2
    params = mlp.init_params(6, np.random.default_rng(6))
    params, losses = mlp.train(params, X, y, np.ones(120), steps=300, lr=3e-3)
    assert losses[-1] < 0.1 * losses[0]
