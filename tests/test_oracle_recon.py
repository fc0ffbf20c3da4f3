"""Oracle pins for the reconstruction driver (L-BFGS, line search, anneal stages) and the
two-point statistics used to score a reconstruction."""
import numpy as np

import synth
from oracle import cosmology as OC
from oracle import lbfgs as LB
from oracle import mesh as M
from oracle import model as OM
from oracle import stats as ST


def _spd(n, seed, lo=1.0, hi=100.0):
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.normal(size=(n, n)))
    return Q @ np.diag(np.geomspace(lo, hi, n)) @ Q.T


def test_two_loop_equals_dense_bfgs_inverse_hessian():
    """The two-loop recursion applies the BFGS-updated inverse Hessian (explicit matrices)."""
    n, m = 9, 5
    A = _spd(n, 1)
    r = np.random.default_rng(2)
    S = [r.normal(size=n) for _ in range(m)]
    Y = [A @ s for s in S]  # curvature s.y > 0
    g = r.normal(size=n)
    H = LB.dense_inverse_hessian(S, Y, n)
    np.testing.assert_allclose(LB.two_loop(g, S, Y), H @ g, rtol=1e-11, atol=1e-12)
    # secant condition of the newest pair: H y = s
    np.testing.assert_allclose(H @ Y[-1], S[-1], rtol=1e-10, atol=1e-12)
    # empty history: H = I
    np.testing.assert_array_equal(LB.two_loop(g, [], []), g)


def test_inner_product_of_complex_modes():
    r = np.random.default_rng(3)
    a = r.normal(size=(4, 4, 3)) + 1j * r.normal(size=(4, 4, 3))
    b = r.normal(size=(4, 4, 3)) + 1j * r.normal(size=(4, 4, 3))
    assert abs(LB.inner(a, b) - np.real(np.vdot(a, b))) < 1e-12
    ra = np.concatenate([a.real.ravel(), a.imag.ravel()])
    rb = np.concatenate([b.real.ravel(), b.imag.ravel()])
    assert abs(LB.inner(a, b) - ra @ rb) < 1e-12


def test_minimize_quadratic_reaches_exact_minimiser():
    n = 30
    A = _spd(n, 4)
    b = np.random.default_rng(5).normal(size=n)
    xs = np.linalg.solve(A, b)

    def fg(x):
        return 0.5 * x @ A @ x - b @ x, A @ x - b

    x, f, info = LB.minimize(fg, np.zeros(n), max_iter=300, rel_tol=0.0)
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
    # every accepted step satisfies the Armijo condition, so the loss never increases
    assert all(b2 <= a2 for a2, b2 in zip(info["losses"], info["losses"][1:]))


def test_minimize_rosenbrock():
    def fg(x):
        a, b = x
        f = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        return f, np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])

    x, f, info = LB.minimize(fg, np.array([-1.2, 1.0]), max_iter=500, rel_tol=0.0)
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-5)


def test_relative_decrease_stopping_rule():
    """A stage stops at the first iteration whose loss decrease is below rel_tol of the loss."""
    A = np.diag([1.0, 1e4])

    def fg(x):
        return 1.0 + 0.5 * x @ A @ x, A @ x

    x, f, info = LB.minimize(fg, np.array([3.0, 2.0]), max_iter=200, rel_tol=1e-3)
    assert info["reason"] == "converged"
    L = info["losses"]
    assert (L[-2] - L[-1]) / L[-2] < 1e-3
    assert all((a - b) / a >= 1e-3 for a, b in zip(L[:-2], L[1:-1]))


def test_power_bins_parseval_and_counts():
    n, box = 16, 100.0
    w = synth.unit_normal(11, (n, n, n))
    a = M.rfft3(w)
    nb = int(np.ceil(np.sqrt(3) * n / 2)) + 1
    cnt, paa, pbb, pab = ST.power_bins(a, a, box, nb)
    assert cnt.sum() == n ** 3 - 1  # every full-spectrum mode but k = 0
    total = np.sum(cnt * paa)
    ref = box ** 3 / n ** 3 * np.sum((w - w.mean()) ** 2)
    assert abs(total - ref) <= 1e-12 * ref
    np.testing.assert_allclose(paa, pab, rtol=1e-14)


def test_power_bins_metrics_special_cases():
    n, box = 16, 100.0
    a = M.rfft3(synth.unit_normal(12, (n, n, n)))
    nb = 8
    cnt, paa, pbb, pab = ST.power_bins(a, a, box, nb)
    full = cnt > 0  # the first shell holds only k = 0, which is excluded
    assert not full[0] and full[1:].all()
    rc, st, tf = ST.metrics(paa, pbb, pab)
    np.testing.assert_allclose(rc[full], 1.0, rtol=1e-14)
    np.testing.assert_allclose(tf[full], 1.0, rtol=1e-14)
    assert np.all(np.abs(st) <= 1e-10 * paa)
    assert rc[0] == 0.0 and tf[0] == 0.0
    _, paa, pbb, pab = ST.power_bins(a, -2.0 * a, box, nb)
    rc, st, tf = ST.metrics(paa, pbb, pab)
    np.testing.assert_allclose(rc[full], -1.0, rtol=1e-14)
    np.testing.assert_allclose(tf[full], 2.0, rtol=1e-14)


def test_power_bins_single_mode_lands_in_its_shell():
    n, box = 16, 100.0
    a = np.zeros((n, n, n // 2 + 1), complex)
    a[3, 4, 0] = 2.0 + 1.0j  # |m| = 5, on the kz = 0 plane (weight 1)
    cnt, paa, _, _ = ST.power_bins(a, a, box, 8)
    assert np.flatnonzero(paa).tolist() == [5]
    assert abs(paa[5] * cnt[5] - box ** 3 / n ** 6 * 5.0) < 1e-15
    # the shell [5, 6) of integer wavevectors, counted by brute force
    m = np.fft.fftfreq(n, 1.0 / n)
    mm = np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2)
    assert cnt[5] == np.count_nonzero((mm >= 5) & (mm < 6))


def test_oracle_reconstruction_recovers_large_scales():
    """L-BFGS on the density-L2 problem (32^3-style setup at 16^3, 3 steps), data from known
    modes, starting from independent modes at 10% power: after 20 iterations the large
    scales are recovered (cross-correlation with the truth near 1, transfer near 1)."""
    n, box = 16, 100.0
    cfg = OM.Config(box, n, n, n, 3, loss_kind=OM.LOSS_DENSITY_L2)
    power = OC.bbks_power()
    inv = OM.prior_inv_variance(n, box, power)
    s_true = OM.linear_modes(synth.white_noise(21, n), box, power)
    target = OM.forward(cfg, s_true, inv, np.zeros((n, n, n)), OM.default_params())["delta_f"]
    s0 = np.sqrt(0.1) * OM.linear_modes(synth.white_noise(22, n), box, power)
    prm = OM.default_params()

    def fg(s):
        fwd, G = OM.gradient(cfg, s, inv, target, prm)
        return fwd["loss"], G

    x, f, info = LB.minimize(fg, s0, max_iter=20, rel_tol=0.0)
    L = info["losses"]
    assert all(b <= a for a, b in zip(L, L[1:])) and L[-1] < 0.2 * L[0]
    rc0, _, _ = ST.metrics(*ST.power_bins(s_true, s0, box, 8)[1:])
    rc, _, tf = ST.metrics(*ST.power_bins(s_true, x, box, 8)[1:])
    assert np.all(rc0[1:4] < 0.3)
    assert np.all(rc[1:4] > 0.95) and np.all(np.abs(tf[1:3] - 1.0) < 0.1)


def test_oracle_anneal_stages_continue_from_previous_optimum():
    """Two log-normal stages (R_sm = 2 then 0): each stage's losses never increase, and the
    second stage starts where the first ended (its first loss is the first stage's optimum
    re-evaluated with the second stage's smoothing)."""
    n, box = 16, 100.0
    cfg = OM.Config(box, n, n, n, 3, loss_kind=OM.LOSS_LOGNORMAL)
    power = OC.bbks_power()
    inv = OM.prior_inv_variance(n, box, power)
    s_true = OM.linear_modes(synth.white_noise(21, n), box, power)
    w = synth.mlp_weights(3, 8)
    target = OM.forward(cfg, s_true, inv, np.ones((n, n, n)), OM.default_params(), w)["mass"]
    s0 = np.sqrt(0.1) * OM.linear_modes(synth.white_noise(22, n), box, power)
    M0 = float(np.median(target))

    def make_fg(R):
        prm = OM.default_params(M0=M0, R_sm=R)

        def fg(s):
            fwd, G = OM.gradient(cfg, s, inv, target, prm, w)
            return fwd["loss"], G
        return fg

    seen = []
    x, infos = LB.reconstruct([2.0, 0.0], make_fg, s0, max_iter=4,
                              log=lambda it, f, t, ev: seen.append(f))
    for info in infos:
        L = info["losses"]
        assert all(b <= a for a, b in zip(L, L[1:]))
    x1 = LB.minimize(make_fg(2.0), s0, max_iter=4)[0]
    assert abs(infos[1]["losses"][0] - make_fg(0.0)(x1)[0]) <= 1e-12 * infos[1]["losses"][0]
