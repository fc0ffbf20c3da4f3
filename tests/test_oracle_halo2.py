"""Oracle pins for the paper's two-network halo model (Sec. 2: model = NNp x NNm;
Sec. 2.1: NNp 81 -> 50 -> 30 -> 1 with ReLU and a sharpened logistic, NNm 3 -> 20 -> 10
-> 1 with ELU and a linear output; Sec. 2.2: NNp sees the three feature fields on the
3 x 3 x 3 neighbourhood of the voxel)."""
import math

import numpy as np
import pytest

import synth
from oracle import cosmology as C
from oracle import mesh as M
from oracle import model as OM


def test_activation_definitions():
    """Eq. elu and Eq. logistic at points where they have closed values."""
    v = np.array([2.0, 1e-300, 0.0, -1.0, -50.0])
    np.testing.assert_allclose(OM.elu(v), [2.0, 1e-300, 0.0, math.exp(-1.0) - 1.0,
                                           math.exp(-50.0) - 1.0], rtol=1e-15, atol=0)
    assert OM.logistic(0.0, 3.0) == 0.5
    assert abs(OM.logistic(1.0, 3.0) - 1.0 / (1.0 + math.exp(-3.0))) < 4e-16
    assert abs(OM.logistic(-0.4, 2.0) - 1.0 / (1.0 + math.exp(0.8))) < 4e-16
    # sharper logistic (larger a) is closer to the step function on both sides
    assert OM.logistic(0.5, 3.0) > OM.logistic(0.5, 1.0)
    assert OM.logistic(-0.5, 3.0) < OM.logistic(-0.5, 1.0)
    with np.errstate(all="raise"):
        assert OM.logistic(-1e4, 3.0) == 0.0 and OM.logistic(1e4, 3.0) == 1.0


def test_stencil_features_brute_force():
    """Feature c * 27 + o at voxel (i, j, k) is field c at (i + dx, j + dy, k + dz) mod n,
    with o running over dx, then dy, then dz in (-1, 0, 1)."""
    n = 5
    f = synth.unit_normal(1, (3, n, n, n))
    F = OM.stencil_features(f)
    assert F.shape == (81, n ** 3)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                v = (i * n + j) * n + k
                o = 0
                for dx in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dz in (-1, 0, 1):
                            for c in range(3):
                                want = f[c, (i + dx) % n, (j + dy) % n, (k + dz) % n]
                                assert F[c * 27 + o, v] == want
                            o += 1
    # the centre of the stencil is the voxel itself
    np.testing.assert_array_equal(F[13], f[0].ravel())


def test_stencil_adjoint_is_the_transpose():
    n = 6
    f = synth.unit_normal(2, (3, n, n, n))
    Fb = synth.unit_normal(3, (81, n ** 3))
    lhs = np.sum(Fb * OM.stencil_features(f))
    rhs = np.sum(OM.stencil_adjoint(Fb, n) * f)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # all-ones adjoint input: every voxel receives 27 contributions per field
    np.testing.assert_allclose(OM.stencil_adjoint(np.ones((81, n ** 3)), n), 27.0)


def test_two_networks_match_explicit_loops():
    """Both networks written neuron by neuron from the architecture, at a few voxels."""
    nets = synth.halo_net_weights(4)
    n, a = 4, 2.0
    f = synth.unit_normal(5, (3, n, n, n))
    out = OM.two_net_forward(nets, f, a)
    P, Mn = nets["nnp"], nets["nnm"]
    for (i, j, k) in [(0, 0, 0), (3, 1, 2), (1, 3, 3)]:
        feats = []
        for c in range(3):
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        feats.append(float(f[c, (i + dx) % n, (j + dy) % n, (k + dz) % n]))
        h1 = [max(0.0, sum(float(P["W1"][u, q]) * feats[q] for q in range(81)) + float(P["b1"][u]))
              for u in range(50)]
        h2 = [max(0.0, sum(float(P["W2"][u, q]) * h1[q] for q in range(50)) + float(P["b2"][u]))
              for u in range(30)]
        y = sum(float(P["W3"][0, q]) * h2[q] for q in range(30)) + float(P["b3"][0])
        pos = 1.0 / (1.0 + math.exp(-a * y))
        x3 = [float(f[c, i, j, k]) for c in range(3)]

        def elu(z):
            return z if z > 0 else math.exp(z) - 1.0
        e1 = [elu(sum(float(Mn["W1"][u, q]) * x3[q] for q in range(3)) + float(Mn["b1"][u]))
              for u in range(20)]
        e2 = [elu(sum(float(Mn["W2"][u, q]) * e1[q] for q in range(20)) + float(Mn["b2"][u]))
              for u in range(10)]
        m = sum(float(Mn["W3"][0, q]) * e2[q] for q in range(10)) + float(Mn["b3"][0])
        v = (i * n + j) * n + k
        assert abs(out["pos"][v] - pos) < 1e-14
        assert abs(out["m"][v] - m) < 1e-13
        assert abs(out["mass"][v] - pos * m) < 1e-13


def test_position_mask_limits():
    """A position network with zero weights and bias outputs 1/2 everywhere (the model is
    half the mass network); with a positive output bias the mask tends to 1 as a grows."""
    nets = synth.halo_net_weights(6)
    n = 4
    f = synth.unit_normal(7, (3, n, n, n))
    z = {k: np.zeros_like(v) for k, v in nets["nnp"].items()}
    out = OM.two_net_forward({"nnp": z, "nnm": nets["nnm"]}, f, 3.0)
    np.testing.assert_array_equal(out["pos"], 0.5)
    np.testing.assert_allclose(out["mass"], 0.5 * out["m"], rtol=1e-15)
    zb = dict(z, b3=np.array([0.4], np.float32))
    p1 = OM.two_net_forward({"nnp": zb, "nnm": nets["nnm"]}, f, 1.0)["pos"]
    p3 = OM.two_net_forward({"nnp": zb, "nnm": nets["nnm"]}, f, 30.0)["pos"]
    assert np.all(p3 > p1) and np.all(p3 > 1.0 - 1e-5)


@pytest.mark.parametrize("a", [1.0, 3.0])
def test_two_net_input_gradient_finite_difference(a):
    """<fbar, df> against central differences of sum(mass_bar * mass(f + eps df)); eps small
    enough that no ReLU changes sign between the two evaluations."""
    nets = synth.halo_net_weights(8)
    n = 6
    f = synth.unit_normal(9, (3, n, n, n))
    mb = synth.unit_normal(10, n ** 3)
    df = synth.unit_normal(11, (3, n, n, n))
    c = OM.two_net_forward(nets, f, a)
    fbar = OM.two_net_backward(nets, c, mb, a, n)
    eps = 1e-7
    cp = OM.two_net_forward(nets, f + eps * df, a)
    cm = OM.two_net_forward(nets, f - eps * df, a)
    for key in ("a1", "a2"):
        assert np.array_equal(cp[key] > 0, cm[key] > 0)
    fd = np.sum(mb * (cp["mass"] - cm["mass"])) / (2 * eps)
    an = np.sum(fbar * df)
    assert abs(fd - an) < 1e-7 * abs(an), (fd, an)


def _setup(n=8, box=40.0, steps=3):
    cfg = OM.Config(box, n, n, n, steps, loss_kind=OM.LOSS_LOGNORMAL, halo_model=OM.HALO_TWO)
    P = C.bbks_power()
    inv = OM.prior_inv_variance(n, box, P)
    s = OM.linear_modes(synth.white_noise(12, n), box, P)
    nets = synth.halo_net_weights(13)
    t = OM.forward(cfg, OM.linear_modes(synth.white_noise(14, n), box, P), inv,
                   np.ones((n,) * 3), OM.default_params(), nets)["mass"]
    return cfg, s, inv, nets, t


@pytest.mark.parametrize("a,R_sm", [(1.0, 2.0), (3.0, 0.0)])
def test_gradient_finite_difference_two_networks(a, R_sm):
    """The mode gradient of the full loss through PM, both networks and the stencil."""
    cfg, s, inv, nets, t = _setup()
    params = OM.default_params(M0=float(np.percentile(t, 60)), R_sm=R_sm, mu=0.1, logistic_a=a)
    _, G = OM.gradient(cfg, s, inv, t, params, nets)
    v = synth.random_modes_direction(15, cfg.n_part) * np.abs(s).mean()
    eps = 1e-6
    fp = OM.forward(cfg, s + eps * v, inv, t, params, nets)
    fm = OM.forward(cfg, s - eps * v, inv, t, params, nets)
    for a_, b_ in zip(fp["xs"], fm["xs"]):
        assert np.array_equal(M.cell_keys(a_, cfg.n_mesh, cfg.box), M.cell_keys(b_, cfg.n_mesh, cfg.box))
    for key in ("a1", "a2"):
        assert np.array_equal(fp["mlp_cache"][key] > 0, fm["mlp_cache"][key] > 0)
    fd = (fp["loss"] - fm["loss"]) / (2 * eps)
    an = np.sum(G.real * v.real + G.imag * v.imag)
    assert abs(fd - an) < 1e-6 * abs(an), (fd, an)


def test_single_network_path_unchanged_by_the_option():
    """halo_model = HALO_SINGLE keeps the softplus network (the default)."""
    cfg = OM.Config(40.0, 8, 8, 8, 2)
    assert cfg.halo_model == OM.HALO_SINGLE
    P = C.bbks_power()
    inv = OM.prior_inv_variance(8, 40.0, P)
    s = OM.linear_modes(synth.white_noise(16, 8), 40.0, P)
    w = synth.mlp_weights(3, 8)
    out = OM.forward(cfg, s, inv, np.ones((8,) * 3), OM.default_params(), w)
    f = OM.features(cfg, out["delta_f"])
    np.testing.assert_array_equal(out["mass"].ravel(), OM.mlp_forward(w, f.reshape(3, -1))["mass"])
