"""Oracle pins for the forward model and its gradient: linear growth, conservation laws,
closed forms of the loss and prior, adjoint identities and finite differences."""
import os

import numpy as np
import pytest

import synth
from oracle import cosmology as C
from oracle import mesh as M
from oracle import model as OM

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_relu_golden():
    with open(os.path.join(GOLDEN, "activations.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                fn, x, v = line.split()
                assert fn == "relu"
                assert OM.relu(np.float64(x)) == np.float64(v)


def test_softplus_and_sigmoid():
    y = np.array([-800.0, -20.0, -1.0, 0.0, 1e-3, 3.0, 40.0, 800.0])
    sp = OM.softplus(y)
    ref = np.array([np.log1p(np.exp(v)) if v < 30 else v + np.log1p(np.exp(-v)) for v in y])
    np.testing.assert_allclose(sp, ref, rtol=1e-15, atol=0)
    assert sp[0] == 0.0 or sp[0] < 1e-300
    h = 1e-6
    fd = (OM.softplus(y[1:-1] + h) - OM.softplus(y[1:-1] - h)) / (2 * h)
    np.testing.assert_allclose(OM.sigmoid(y[1:-1]), fd, rtol=1e-8, atol=1e-12)


def test_prior_of_generated_field_is_half_the_white_noise_energy():
    """s = rfft(w) sqrt(n^3 P / L^3) and 1/S = L^3 / (n^6 P) make the prior exponent
    0.5 sum_full |s|^2 / S equal 0.5 (sum w^2 - (sum w)^2 / n^3) exactly (Parseval)."""
    n, box = 16, 100.0
    P = C.bbks_power()
    w = synth.white_noise(11, n)
    s = OM.linear_modes(w, box, P)
    inv = OM.prior_inv_variance(n, box, P)
    lp = OM.prior_loss(s, inv)
    expect = 0.5 * (np.sum(w * w) - np.sum(w) ** 2 / n ** 3)
    assert abs(lp - expect) < 1e-10 * expect


def test_perfect_lattice_feels_no_force():
    cfg = OM.Config(40.0, 8, 16, 8, 1)
    q = M.lattice_positions(8, 40.0, 16)
    d = OM.density(cfg, q, 16)
    np.testing.assert_allclose(d, 0.0, atol=1e-13)
    F = OM.force_meshes(cfg, d)
    assert np.abs(F).max() < 1e-13


def test_zero_modes_keep_the_lattice_exactly():
    """An empty linear field through the whole forward model: with L = 32 on an 16^3
    lattice and mesh every CIC fraction is exactly 1/2, so the density is exactly uniform,
    the force exactly zero, and every position stays on its lattice site bit for bit."""
    n = 16
    cfg = OM.Config(32.0, n, n, n, 3, loss_kind=OM.LOSS_LOGNORMAL)
    P = C.bbks_power()
    inv = OM.prior_inv_variance(n, 32.0, P)
    s = np.zeros_like(OM.linear_modes(synth.white_noise(3, n), 32.0, P))
    out = OM.forward(cfg, s, inv, np.ones((n,) * 3), OM.default_params(), synth.mlp_weights(3, 8))
    q = M.lattice_positions(n, 32.0, n)
    for x in out["xs"]:
        assert np.array_equal(x, q)
    assert np.all(out["delta_f"] == 0.0) and out["loss_prior"] == 0.0
    # the network then sees zero features everywhere: one mass value for every voxel
    assert np.all(out["mass"] == out["mass"].ravel()[0])


def test_total_momentum_is_conserved():
    """CIC both ways with an odd force kernel: sum_p F(x_p) = rho^T A rho = 0."""
    n, box = 16, 50.0
    cfg = OM.Config(box, 8, n, 8, 1)
    x = synth.random_positions(21, 8 ** 3, box)
    F = OM.force_meshes(cfg, OM.density(cfg, x, n))
    Fp = M.cic_readout(x, n, box, F)
    scale = np.abs(Fp).sum()
    assert np.all(np.abs(Fp.sum(axis=1)) < 1e-12 * scale)


def _single_mode_modes(n, box, m, amp):
    """Stored modes of the linear field delta_L = amp cos(k.q)."""
    g = np.arange(n) * box / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    k = 2 * np.pi * np.array(m) / box
    return M.rfft3(amp * np.cos(k[0] * X + k[1] * Y + k[2] * Z)), k


def _linear_growth_error(n):
    box = 100.0
    s, k = _single_mode_modes(n, box, (1, 0, 0), 1e-3)
    cfg = OM.Config(box, n, n, n, 5)
    x0, p0, psi = OM.zeldovich(cfg, s)
    xs, *_ = OM.pm_forward(cfg, x0, p0)
    q = M.lattice_positions(n, box, n)
    disp = (xs[-1] - q + box / 2) % box - box / 2
    expect = C.growth_D(1.0, cfg.omega_m) * psi
    return np.abs(disp - expect).max() / np.abs(expect).max()


def test_pm_follows_linear_growth_on_large_scales():
    """A single low-k mode of small amplitude: after the full evolution every particle sits
    at q + D(1) Psi(q) (Zel'dovich, Sec. 3) up to the CIC window, whose error is
    (k dx)^2 / 6 and so falls four-fold when the resolution doubles."""
    e16, e32 = _linear_growth_error(16), _linear_growth_error(32)
    kdx = 2 * np.pi / 16
    assert e16 < 1.1 * kdx ** 2 / 6
    assert 3.6 < e16 / e32 < 4.4


def test_zeldovich_displacement_divergence():
    """Psi = i k delta / k^2 gives div Psi = -delta_L for a single mode."""
    n, box = 16, 64.0
    s, k = _single_mode_modes(n, box, (1, 2, 0), 0.01)
    cfg = OM.Config(box, n, n, n, 1)
    _, _, psi = OM.zeldovich(cfg, s)
    g = np.arange(n) * box / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    ph = (k[0] * X + k[1] * Y + k[2] * Z).ravel()
    for a in range(3):
        np.testing.assert_allclose(psi[a], -0.01 * k[a] / (k @ k) * np.sin(ph), atol=1e-15)


@pytest.mark.parametrize("m", [(1, 0, 0), (0, 2, 1), (3, -1, 2)])
def test_features_single_mode_closed_form(m):
    """Sec. 2.2 features of a single Fourier mode: for delta = A cos(k.x) on the mesh nodes,
    a Gaussian smoothing on R multiplies it by exp(-k^2 R^2 / 2), so the three features are
    (A cos, g1 A cos, (g1 - g2) A cos) with g_j = exp(-k^2 R_j^2 / 2). Written with the
    trigonometric form directly (no FFT), so a swapped, dropped or mis-signed feature, or
    a wrong k scaling in the multiplier, fails."""
    n, box, A = 16, 50.0, 0.7
    cfg = OM.Config(box, n, n, n, 1, R1=1.5, R2=4.0)
    i = np.arange(n) * (box / n)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    k = 2 * np.pi * np.array(m) / box
    base = A * np.cos(k[0] * X + k[1] * Y + k[2] * Z)
    k2 = float(k @ k)
    g1, g2 = np.exp(-0.5 * k2 * cfg.R1 ** 2), np.exp(-0.5 * k2 * cfg.R2 ** 2)
    f = OM.features(cfg, base)
    assert f.shape == (3, n, n, n)
    np.testing.assert_allclose(f[0], base, rtol=0, atol=1e-13)
    np.testing.assert_allclose(f[1], g1 * base, rtol=0, atol=1e-13)
    np.testing.assert_allclose(f[2], (g1 - g2) * base, rtol=0, atol=1e-13)
    # the two smoothings differ measurably at these scales, so f[2] != f[1] and != g2 base
    assert abs(g1 - g2) > 1e-2 and g2 > 1e-3


def test_mlp_matches_explicit_loops():
    w = synth.mlp_weights(3, 6)
    f = synth.unit_normal(4, (3, 5))
    out = OM.mlp_forward(w, f)
    for v in range(5):
        h1 = [max(0.0, sum(float(w["W1"][j, i]) * f[i, v] for i in range(3)) + float(w["b1"][j]))
              for j in range(6)]
        h2 = [max(0.0, sum(float(w["W2"][j, i]) * h1[i] for i in range(6)) + float(w["b2"][j]))
              for j in range(6)]
        y = sum(float(w["W3"][0, i]) * h2[i] for i in range(6)) + float(w["b3"][0])
        assert abs(out["mass"][v] - np.log1p(np.exp(y))) < 1e-14


def _setup(n=16, box=50.0, steps=3, kind=OM.LOSS_LOGNORMAL, hidden=8):
    cfg = OM.Config(box, n, n, n, steps, loss_kind=kind)
    P = C.bbks_power()
    inv = OM.prior_inv_variance(n, box, P)
    s = OM.linear_modes(synth.white_noise(1, n), box, P)
    w = synth.mlp_weights(3, hidden) if kind == OM.LOSS_LOGNORMAL else None
    s2 = OM.linear_modes(synth.white_noise(2, n), box, P)
    if kind == OM.LOSS_LOGNORMAL:
        t = OM.forward(cfg, s2, inv, np.ones((n,) * 3), OM.default_params(), w)["mass"]
    else:
        t = OM.forward(cfg, s2, inv, np.zeros((n,) * 3), OM.default_params())["delta_f"]
    return cfg, s, inv, w, t


@pytest.mark.parametrize("R_sm", [0.0, 1.0, 4.0])
def test_loss_closed_form_when_model_equals_data(R_sm):
    """With the model's own mass as data the residual is the constant mu / (2 sigma_N),
    which the smoothing leaves alone: L_data = N^3 (mu / 2 sigma_N)^2 (Eq. loss)."""
    cfg, s, inv, w, _ = _setup()
    mass = OM.forward(cfg, s, inv, np.ones((16,) * 3), OM.default_params(), w)["mass"]
    pr = OM.default_params(mu=0.3, sigma_N=0.5, M0=0.7, R_sm=R_sm)
    out = OM.forward(cfg, s, inv, mass, pr, w)
    assert abs(out["loss_data"] - 16 ** 3 * (0.3 / 1.0) ** 2) < 1e-9 * out["loss_data"]
    # mu = 0: zero data gradient, the gradient is the prior's alone
    pr0 = OM.default_params(mu=0.0, M0=0.7, R_sm=R_sm)
    _, G = OM.gradient(cfg, s, inv, mass, pr0, w)
    np.testing.assert_allclose(G, OM.prior_grad(s, inv), atol=1e-12 * np.abs(G).max())


def _dot_test(fwd_op, adj_op, x, y):
    lhs = np.vdot(fwd_op(x).ravel(), y.ravel()).real
    rhs = np.vdot(x.ravel(), adj_op(y).ravel()).real
    assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), 1e-300)


def test_force_operator_adjoint():
    n, box = 16, 40.0
    cfg = OM.Config(box, 8, n, 8, 1)
    d = synth.unit_normal(1, (n, n, n))
    Fb = synth.unit_normal(2, (3, n, n, n))
    _dot_test(lambda v: OM.force_meshes(cfg, v), lambda u: OM.force_adjoint_mesh(cfg, u), d, Fb)


def test_zeldovich_adjoint_identity():
    """<Psi(s), u> = sum_stored Re(G) Re(s) + Im(G) Im(s) with G the adjoint of u."""
    n, box = 8, 30.0
    cfg = OM.Config(box, n, n, n, 1)
    s = synth.random_modes_direction(3, n)
    u = synth.unit_normal(4, (3, n ** 3))
    _, _, psi = OM.zeldovich(cfg, s)
    lhs = np.sum(psi * u)
    G = OM.zeldovich_adjoint(cfg, u / cfg.fac["D0"], 0 * u)
    rhs = np.sum(G.real * s.real + G.imag * s.imag)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def _fd_check(cfg, s, inv, t, params, w, seed, eps=1e-6, tol=1e-6):
    """Central difference along a random direction; eps is chosen small enough that no
    particle changes cell between the two evaluations (CIC has kinks at cell faces)."""
    _, G = OM.gradient(cfg, s, inv, t, params, w)
    v = synth.random_modes_direction(seed, cfg.n_part) * np.abs(s).mean()
    fp = OM.forward(cfg, s + eps * v, inv, t, params, w)
    fm = OM.forward(cfg, s - eps * v, inv, t, params, w)
    changes = sum(int(np.sum(M.cell_keys(a, cfg.n_mesh, cfg.box) != M.cell_keys(b, cfg.n_mesh, cfg.box)))
                  for a, b in zip(fp["xs"], fm["xs"]))
    assert changes == 0
    fd = (fp["loss"] - fm["loss"]) / (2 * eps)
    an = np.sum(G.real * v.real + G.imag * v.imag)
    assert abs(fd - an) < tol * abs(an), (fd, an)


@pytest.mark.parametrize("R_sm", [0.0, 2.0])
def test_gradient_finite_difference_lognormal(R_sm):
    cfg, s, inv, w, t = _setup()
    params = OM.default_params(M0=float(np.percentile(t, 50)), R_sm=R_sm, mu=0.1)
    _fd_check(cfg, s, inv, t, params, w, seed=5)


def test_gradient_finite_difference_density_l2_small_box():
    """Density-L2 loss against a target from a second seed (32^3, L = 100, 5 steps)."""
    cfg, s, inv, _, t = _setup(n=32, box=100.0, steps=5, kind=OM.LOSS_DENSITY_L2)
    _fd_check(cfg, s, inv, t, OM.default_params(prior_weight=0.0), None, seed=6)


def test_gradient_finite_difference_force_mesh_twice_particles():
    """Force mesh at twice the particle resolution (the larger-mesh configuration)."""
    n, box = 8, 40.0
    cfg = OM.Config(box, n, 2 * n, n, 3, loss_kind=OM.LOSS_LOGNORMAL)
    P = C.bbks_power()
    inv = OM.prior_inv_variance(n, box, P)
    s = OM.linear_modes(synth.white_noise(8, n), box, P)
    w = synth.mlp_weights(9, 4)
    t = OM.forward(cfg, OM.linear_modes(synth.white_noise(10, n), box, P), inv,
                   np.ones((n,) * 3), OM.default_params(), w)["mass"]
    params = OM.default_params(M0=float(np.percentile(t, 75)), R_sm=1.0)
    _fd_check(cfg, s, inv, t, params, w, seed=11)


# ------------------------------------------------------------------ mass-dependent noise

def _table_around(t, mu=(0.3, -0.1, 0.2), sig=(0.8, 0.4, 0.6)):
    """Three interpolation nodes spanning the 10th-90th percentile of log(M_R,data)."""
    lo, mid, hi = np.percentile(t, [10, 50, 90])
    return (np.array([lo, mid, hi]), np.array(mu), np.array(sig))


def _logmr(cfg, target, params):
    with np.errstate(divide="ignore"):
        return np.log(np.maximum(OM.smooth(cfg, target, params["R_mass"]), 0.0))


def test_noise_table_constant_equals_scalar_model():
    cfg, s, inv, w, t = _setup()
    base = OM.default_params(M0=float(np.percentile(t, 50)), mu=0.1, sigma_N=0.7, R_sm=2.0)
    tab = dict(base, noise_table=([-3.0, 0.0, 2.0], [0.1] * 3, [0.7] * 3))
    a, Ga = OM.gradient(cfg, s, inv, t, base, w)
    b, Gb = OM.gradient(cfg, s, inv, t, tab, w)
    assert a["loss"] == b["loss"]
    np.testing.assert_array_equal(Ga, Gb)


def test_noise_table_clamps_to_end_nodes():
    """Nodes all below (above) every cell's log(M_R,data): every cell takes the last (first)
    node's values, i.e. the scalar model with those values."""
    cfg, s, inv, w, t = _setup()
    base = OM.default_params(M0=float(np.percentile(t, 50)), R_sm=0.0)
    lm = _logmr(cfg, t, base)
    lo, hi = lm.min(), lm.max()
    below = dict(base, noise_table=([lo - 3, lo - 2], [0.5, 0.2], [0.9, 0.3]))
    above = dict(base, noise_table=([hi + 1, hi + 2], [0.5, 0.2], [0.9, 0.3]))
    fb = OM.forward(cfg, s, inv, t, below, w)["loss"]
    fa = OM.forward(cfg, s, inv, t, above, w)["loss"]
    assert fb == OM.forward(cfg, s, inv, t, dict(base, mu=0.2, sigma_N=0.3), w)["loss"]
    assert fa == OM.forward(cfg, s, inv, t, dict(base, mu=0.5, sigma_N=0.9), w)["loss"]


def test_noise_table_width_scaling():
    """Scaling every sigma node by lam (mu = 0) scales the data term and its gradient by
    1 / lam^2: the width enters the residual once and its adjoint once."""
    cfg, s, inv, w, t = _setup()
    base = OM.default_params(M0=float(np.percentile(t, 50)), R_sm=1.0, prior_weight=0.0)
    nodes, _, sig = _table_around(_logmr(cfg, t, base))
    p1 = dict(base, noise_table=(nodes, [0.0] * 3, sig))
    p2 = dict(base, noise_table=(nodes, [0.0] * 3, 2.5 * sig))
    a, Ga = OM.gradient(cfg, s, inv, t, p1, w)
    b, Gb = OM.gradient(cfg, s, inv, t, p2, w)
    assert abs(b["loss"] * 2.5 ** 2 - a["loss"]) <= 1e-12 * a["loss"]
    np.testing.assert_allclose(Gb * 2.5 ** 2, Ga, rtol=1e-10, atol=1e-12 * np.abs(Ga).max())


def test_noise_table_loss_at_model_equals_data():
    """Model = data: x_model = x_data, so the data term is sum (mu_i / (2 sigma_i))^2 with
    R_sm = 0, where the nodes' own values are taken at cells whose log(M_R,data) is a node."""
    cfg, s, inv, w, _ = _setup()
    t = OM.forward(cfg, s, inv, np.ones((cfg.n_out,) * 3), OM.default_params(), w)["mass"]
    base = OM.default_params(M0=float(np.percentile(t, 50)), R_sm=0.0)
    lm = _logmr(cfg, t, base).ravel()
    # nodes at the exact values of three cells
    idx = np.argsort(lm)[[len(lm) // 10, len(lm) // 2, 9 * len(lm) // 10]]
    nodes = lm[idx]
    mu, sig = np.array([0.3, -0.1, 0.2]), np.array([0.8, 0.4, 0.6])
    p = dict(base, noise_table=(nodes, mu, sig))
    mu_i, sig_i = OM.noise_fields(cfg, t, p)
    np.testing.assert_array_equal(mu_i.ravel()[idx], mu)
    np.testing.assert_array_equal(sig_i.ravel()[idx], sig)
    f = OM.forward(cfg, s, inv, t, p, w)
    assert abs(f["loss_data"] - np.sum((mu_i / (2 * sig_i)) ** 2)) <= 1e-12 * f["loss_data"]


def test_gradient_finite_difference_noise_table():
    cfg, s, inv, w, t = _setup()
    base = OM.default_params(M0=float(np.percentile(t, 50)), R_sm=2.0)
    params = dict(base, noise_table=_table_around(_logmr(cfg, t, base)))
    _fd_check(cfg, s, inv, t, params, w, seed=12)


# ------------------------------------------------------------------ second-order LPT

def _plane_wave_modes(n, waves):
    """Half spectrum of sum_j A_j cos(2 pi m_j . q / n) on the lattice (exact)."""
    g = np.indices((n, n, n)).reshape(3, -1).T
    f = np.zeros(n ** 3)
    for A, m in waves:
        f += A * np.cos(2 * np.pi * (g @ np.asarray(m, float)) / n)
    return M.rfft3(f.reshape(n, n, n))


def test_lpt2_single_plane_wave_equals_zeldovich():
    """A one-dimensional perturbation has no second-order source: 2LPT = Zel'dovich."""
    n, box = 16, 50.0
    s = _plane_wave_modes(n, [(30.0, (2, 0, 0))])
    c1 = OM.Config(box, n, n, n, 3, ic_order=1)
    c2 = OM.Config(box, n, n, n, 3, ic_order=2)
    x1, p1, _ = OM.zeldovich(c1, s)
    x2, p2, _, ex = OM.zeldovich(c2, s, full=True)
    assert np.abs(ex["S"]).max() < 1e-10 * 30.0 ** 2
    np.testing.assert_allclose(x2, x1, rtol=0, atol=1e-12 * box)
    np.testing.assert_allclose(p2, p1, rtol=0, atol=1e-12 * np.abs(p1).max())


def test_lpt2_two_crossed_plane_waves_closed_form():
    """delta = A cos(k1 x) + B cos(k2 y): phi_xx = A cos(k1 x), phi_yy = B cos(k2 y), the other
    second derivatives vanish, so S = A B cos(k1 x) cos(k2 y) and
    Psi2 = -A B (k1 sin(k1 x) cos(k2 y), k2 cos(k1 x) sin(k2 y), 0) / (k1^2 + k2^2)."""
    n, box = 16, 50.0
    A, B, m1, m2 = 3.0, 2.0, 2, 3
    s = _plane_wave_modes(n, [(A, (m1, 0, 0)), (B, (0, m2, 0))])
    cfg = OM.Config(box, n, n, n, 3, ic_order=2)
    _, _, _, ex = OM.zeldovich(cfg, s, full=True)
    i, j, _ = np.indices((n, n, n))
    cx, sx = np.cos(2 * np.pi * m1 * i / n), np.sin(2 * np.pi * m1 * i / n)
    cy, sy = np.cos(2 * np.pi * m2 * j / n), np.sin(2 * np.pi * m2 * j / n)
    np.testing.assert_allclose(ex["phi"][0], A * cx, atol=1e-12)
    np.testing.assert_allclose(ex["phi"][1], B * cy, atol=1e-12)
    for k in (2, 3, 4, 5):
        assert np.abs(ex["phi"][k]).max() < 1e-12
    np.testing.assert_allclose(ex["S"], A * B * cx * cy, atol=1e-11)
    k1, k2 = 2 * np.pi * m1 / box, 2 * np.pi * m2 / box
    ref = -A * B / (k1 ** 2 + k2 ** 2) * np.stack([k1 * sx * cy, k2 * cx * sy, 0 * cx])
    np.testing.assert_allclose(ex["psi2"], ref.reshape(3, -1), atol=1e-12)


def test_lpt2_term_is_quadratic_in_the_modes():
    cfg, s, inv, w, t = _setup()
    c2 = OM.Config(cfg.box, cfg.n_part, cfg.n_mesh, cfg.n_out, 3, ic_order=2)
    _, _, _, e1 = OM.zeldovich(c2, s, full=True)
    _, _, _, e3 = OM.zeldovich(c2, 3.0 * s, full=True)
    np.testing.assert_allclose(e3["psi2"], 9.0 * e1["psi2"], rtol=1e-10,
                               atol=1e-12 * np.abs(e3["psi2"]).max())


def test_gradient_finite_difference_lpt2():
    cfg, s, inv, w, t = _setup()
    c2 = OM.Config(cfg.box, cfg.n_part, cfg.n_mesh, cfg.n_out, cfg.n_steps, ic_order=2)
    params = OM.default_params(M0=float(np.percentile(t, 50)), R_sm=1.0, mu=0.1)
    _fd_check(c2, s, inv, t, params, w, seed=13)


def test_gradient_finite_difference_lpt2_density_l2():
    cfg, s, inv, _, t = _setup(n=16, box=50.0, steps=3, kind=OM.LOSS_DENSITY_L2)
    c2 = OM.Config(cfg.box, cfg.n_part, cfg.n_mesh, cfg.n_out, cfg.n_steps,
                   loss_kind=OM.LOSS_DENSITY_L2, ic_order=2)
    _fd_check(c2, s, inv, t, OM.default_params(prior_weight=0.0), None, seed=14)
