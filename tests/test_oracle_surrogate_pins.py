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


# ---------------------------------------------------------------- wedge, star map, features, gate
from oracle import linewidths as olw  # noqa: E402
from oracle import surrogate as osur  # noqa: E402


@pytest.mark.parametrize("n,count", [(4, 8), (6, 16), (8, 29)])
def test_fcc_wedge_counts_match_textbook(n, count):
    """Gamma-centred n^3 meshes of an fcc crystal with the full cubic group
    have 8, 16 and 29 irreducible points (standard k-point tables)."""
    ir = osur.ibz_map(models.diamond(), (n, n, n))
    assert len(np.unique(ir)) == count
    assert osur.star_sizes(ir).sum() == n ** 3


@pytest.mark.parametrize("n", [4, 6])
def test_simple_cubic_wedge_closed_form(n):
    """Simple cubic, even n: the wedge 0 <= z <= y <= x <= n/2 holds
    (n/2+1)(n/2+2)(n/2+3)/6 points."""
    ir = osur.ibz_map(models.perovskite(0), (n, n, n))
    h = n // 2
    assert len(np.unique(ir)) == (h + 1) * (h + 2) * (h + 3) // 6


@pytest.mark.parametrize("which", ["diamond", "perovskite", "random"])
def test_crystal_operations_form_a_group(which):
    """The operations found hold the identity and are closed under products
    and inverses; the cubic crystals keep all 48."""
    m = {"diamond": models.diamond(), "perovskite": models.perovskite(0),
         "random": models.random_cell(5, 2)}[which]
    ops = osur.crystal_operations(m)
    key = lambda R: tuple(np.rint(R).astype(int).reshape(-1))
    have = {key(R) for R in ops}
    assert key(np.eye(3)) in have
    for A in ops:
        assert key(A.T) in have
        for B in ops:
            assert key(A @ B) in have
    if which != "random":
        assert len(ops) == 48


def test_star_members_share_frequencies_and_jdos():
    """Point symmetry of the dynamics: every q of a star has the spectrum of
    its representative, and the phase space D+- is a function of the star."""
    m = models.diamond()
    mesh = (4, 4, 4)
    ir = osur.ibz_map(m, mesh)
    om, ev, ve = phonons.phonons(m, mesh)
    # zero-frequency branches of the nearest-neighbour model carry eigen-solver noise
    np.testing.assert_allclose(om, om[ir], rtol=1e-10, atol=1e-4)
    # fixed width: adaptive widths use partner velocities, whose split inside a
    # degenerate multiplet follows a gauge that is not point-symmetric
    dp, dm = ojdos.jdos(m, mesh, om, ve, B_FIXED)
    np.testing.assert_allclose(dp, dp[ir], rtol=1e-8, atol=1e-12 * dp.max())
    np.testing.assert_allclose(dm, dm[ir], rtol=1e-8, atol=1e-12 * dm.max())


@pytest.mark.parametrize("which", ["diamond", "perovskite"])
def test_star_map_reproduces_full_mesh_linewidths(which):
    """Gamma computed on every q equals, after averaging over degenerate
    clusters, the star map of the representatives' values, and the
    representatives alone (a q_list of the wedge) give the same map."""
    m = models.diamond() if which == "diamond" else models.perovskite(0)
    mesh = (4, 4, 4)
    ir = osur.ibz_map(m, mesh)
    om, ev, ve = phonons.phonons(m, mesh)
    g = olw.crystal_linewidths(m, mesh, om, ev, ve, 300.0, B_FIXED)
    mapped = osur.star_map(ir, om, g)
    own = osur.star_map(np.arange(len(ir)), om, g)   # cluster averages at each q itself
    scale = g.max()
    np.testing.assert_allclose(mapped, own, rtol=1e-7, atol=1e-9 * scale)
    g_ir = olw.crystal_linewidths(m, mesh, om, ev, ve, 300.0, B_FIXED, q_list=np.unique(ir))
    np.testing.assert_allclose(osur.star_map(ir, om, g_ir), own, rtol=1e-7, atol=1e-9 * scale)


def test_features_are_star_invariant():
    m = models.diamond()
    mesh = (4, 4, 4)
    ir = osur.ibz_map(m, mesh)
    om, ev, ve = phonons.phonons(m, mesh)
    dp, dm = ojdos.jdos(m, mesh, om, ve, B_FIXED)
    nb3 = om.shape[1]
    modes = np.arange(om.size)
    F = osur.features(m, mesh, om, ve, dp, dm, modes)
    Fr = osur.features(m, mesh, om, ve, dp, dm, (ir[modes // nb3] * nb3 + modes % nb3))
    cols = [0] + list(range(2 + nb3, nb3 + 8))  # nu, q components, |q|, ln(1 + D)
    np.testing.assert_allclose(F[:, cols], Fr[:, cols], rtol=1e-8, atol=1e-5)  # zero-branch noise
    # |q| of the shortest image never exceeds the image at the mesh coordinates
    B = phonons.reciprocal(m.lattice)
    q0 = (phonons.mesh_points(mesh) / np.asarray(mesh)) @ B
    assert np.all(F[:, nb3 + 5] <= np.linalg.norm(q0, axis=1)[modes // nb3] + 1e-12)


def test_standardize_moments():
    X = np.random.default_rng(3).normal(2.0, 3.0, size=(50, 4))
    X[:, 2] = 5.0
    Z, mu, sd = osur.standardize(X, 30)
    np.testing.assert_allclose(Z[:30, [0, 1, 3]].mean(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose(Z[:30, [0, 1, 3]].std(axis=0), 1.0, rtol=1e-12)
    assert sd[2] == 1.0 and np.all(Z[:, 2] == 0.0)


def test_gate_threshold_small_cases():
    gt = np.array([1.0, 1.0, 1.0, 1.0])
    w = np.ones(4)
    sp = np.array([0.1, 0.2, 0.3, 0.4], np.float32)
    # perfect predictions: every row accepted
    tau = osur.gate_threshold(gt, gt.copy(), sp, w, 0.0)
    assert tau == np.nextafter(np.float32(0.4), np.float32(np.inf))
    # row with spread 0.2 off by 1/G: +1 on a reference sum of 4 -> needs tol >= 0.25
    gp = np.array([1.0, 0.5, 1.0, 1.0])
    assert osur.gate_threshold(gt, gp, sp, w, 0.24) == np.nextafter(np.float32(0.1), np.float32(np.inf))
    assert osur.gate_threshold(gt, gp, sp, w, 0.25) == np.nextafter(np.float32(0.4), np.float32(np.inf))
    # a bad first row accepts nothing
    gp = np.array([0.5, 1.0, 1.0, 1.0])
    assert osur.gate_threshold(gt, gp, sp, w, 0.1) == 0.0
    # tied spreads are one group
    sp2 = np.array([0.1, 0.1, 0.3, 0.4], np.float32)
    gp = np.array([1.0, 0.5, 1.0, 1.0])
    assert osur.gate_threshold(gt, gp, sp2, w, 0.24) == 0.0
    # an error that a later row cancels is still a stop (prefix rule)
    gp = np.array([1.0, 0.5, 2.0, 1.0])
    assert osur.gate_threshold(gt, gp, sp, w, 0.2) == np.nextafter(np.float32(0.1), np.float32(np.inf))


def test_gate_score_is_first_order_kappa_error():
    """score = |d(w/Gamma)| for a shift of ln Gamma by spread*sd, to first order."""
    w = np.array([2.0, 5.0, 0.3])
    mean = np.array([0.1, -0.4, 1.2])
    y_mu_sd = (-1.0, 0.7)
    spread = np.array([1e-6, 2e-6, 3e-6])
    s = osur.gate_score(mean, spread, y_mu_sd, w)
    l = mean * y_mu_sd[1] + y_mu_sd[0]
    exact = np.abs(w / np.exp(l + spread * y_mu_sd[1]) - w / np.exp(l))
    np.testing.assert_allclose(s, exact, rtol=1e-5)
    inside = np.array([True, False, True])
    assert np.isinf(osur.gate_score(mean, spread, y_mu_sd, w, inside)[1])
