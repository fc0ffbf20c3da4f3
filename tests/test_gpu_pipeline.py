"""End-to-end GPU parity: forward model, loss and mode gradient against the FP64 oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import cosmology as OC
from oracle import mesh as M
from oracle import model as OM
import paper_1805_02247_amd as P
from _gpu import DEV, cosine, rel_l2, require_gpu, say

pytestmark = pytest.mark.gpu


def _problem(n, nm, no, box, steps, kind, B, hidden=8, R_sm=(0.0,), seed=1, mu=0.1,
             prior_weight=1.0, ic_order=1):
    ocfg = OM.Config(box, n, nm, no, steps, loss_kind=kind, ic_order=ic_order)
    power = OC.bbks_power()
    inv = OM.prior_inv_variance(n, box, power)
    modes = [OM.linear_modes(synth.white_noise(seed + 10 * b, n), box, power) for b in range(B)]
    w = synth.mlp_weights(3, hidden) if kind == OM.LOSS_LOGNORMAL else None
    targets, params = [], []
    for b in range(B):
        st = OM.linear_modes(synth.white_noise(seed + 10 * b + 5, n), box, power)
        if kind == OM.LOSS_LOGNORMAL:
            t = OM.forward(ocfg, st, inv, np.ones((no,) * 3), OM.default_params(), w)["mass"]
            prm = OM.default_params(M0=float(np.percentile(t, 50)), R_sm=R_sm[b % len(R_sm)], mu=mu,
                                    prior_weight=prior_weight)
        else:
            t = OM.forward(ocfg, st, inv, np.zeros((no,) * 3), OM.default_params())["delta_f"]
            prm = OM.default_params(prior_weight=0.0)
        targets.append(t)
        params.append(prm)
    return ocfg, inv, modes, w, targets, params


def _gpu_run(ocfg, inv, modes, w, targets, params, hidden=8, ckpt=0, precision=P.PMR_FP32,
             noise=None):
    B = len(modes)
    n = ocfg.n_part
    cfg = P.Config(batch=B, n_part=n, n_mesh=ocfg.n_mesh, n_out=ocfg.n_out, n_steps=ocfg.n_steps,
                   mlp_hidden=hidden, box=ocfg.box, ckpt_every=ckpt, precision=precision,
                   loss_kind=ocfg.loss_kind, R1=ocfg.R1, R2=ocfg.R2, ic_order=ocfg.ic_order,
                   halo_model=ocfg.halo_model)
    pm = P.PMContext(cfg, DEV)
    pm.set_prior(torch.from_numpy(inv.astype(np.float32)))
    if w is not None and ocfg.halo_model == OM.HALO_TWO:
        pm.set_halo_nets(w)
    elif w is not None:
        pm.set_mlp({k: torch.from_numpy(v) for k, v in w.items()})
    pm.set_target(torch.from_numpy(np.stack(targets).astype(np.float32)).reshape(B, -1))
    pm.set_loss([P.LossParams(**{k: v for k, v in p.items() if k != "noise_table"})
                 for p in params])
    if noise is not None:
        pm.set_noise_table(*noise)
    m = torch.from_numpy(np.stack(modes).astype(np.complex64)).reshape(B, -1).to(DEV)
    mass, loss = pm.forward(m)
    xs = [pm.debug("x", i).cpu().numpy() for i in range(ocfg.n_steps + 1)] if ckpt == 0 else None
    delta_f = pm.debug("delta_f").cpu().numpy()
    g = pm.adjoint(torch.ones(B, dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    return dict(pm=pm, mass=mass.cpu().numpy(), loss=loss.cpu().numpy(), xs=xs,
                delta_f=delta_f, grad=g.cpu().numpy(), xbar0=pm.debug("xbar0").cpu().numpy(),
                modes=m)


def _compare(ocfg, inv, modes, w, targets, params, res, tol, refs=None):
    B = len(modes)
    for b in range(B):
        if refs is None:
            ref, G = OM.gradient(ocfg, modes[b], inv, targets[b], params[b], w)
        else:
            ref, G = refs[b]
        out = {}
        if res["xs"] is not None:
            dx = 0.0
            for i, xr in enumerate(ref["xs"]):
                d = res["xs"][i][b] - xr
                d = (d + ocfg.box / 2) % ocfg.box - ocfg.box / 2
                dx = max(dx, np.abs(d).max() / (ocfg.box / ocfg.n_mesh))
            out["max_dx_cells"] = dx
            # particles whose final CIC cell differs from the oracle's (reported, not failed:
            # a position within rounding of a cell face may land on either side)
            h = ocfg.box / ocfg.n_mesh
            cg = np.floor(res["xs"][-1][b] / h).astype(np.int64) % ocfg.n_mesh
            cr = np.floor(ref["xs"][-1] / h).astype(np.int64) % ocfg.n_mesh
            out["cell_flips"] = float(np.any(cg != cr, axis=0).sum())
        out["delta_f"] = rel_l2(res["delta_f"][b], ref["delta_f"].ravel())
        out["loss"] = abs(res["loss"][b, 0] - ref["loss"]) / abs(ref["loss"])
        dp = abs(res["loss"][b, 1] - ref["loss_prior"])
        out["prior"] = dp / abs(ref["loss_prior"]) if ref["loss_prior"] != 0 else dp
        g = res["grad"][b].reshape(G.shape)
        out["grad_cos"] = cosine(g, G)
        out["grad_rel"] = rel_l2(g, G)
        if ref.get("mass") is not None:
            out["mass"] = rel_l2(res["mass"][b], ref["mass"].ravel())
        say(f"  item {b}: " + ", ".join(f"{k}={v:.3e}" for k, v in out.items()))
        for k, lim in tol.items():
            if k == "grad_cos":
                assert out[k] >= lim, (k, out[k])
            elif k in out:
                assert out[k] <= lim, (k, out[k])


# FP32 path against the FP64 oracle (measured: loss <= 5e-7, gradient rel-L2 <= 2.3e-5 on
# every case below except the two small two-network meshes).
TOL_FP32 = {"max_dx_cells": 1e-4, "delta_f": 1e-4, "loss": 1e-5, "prior": 1e-5, "mass": 1e-4,
            "grad_cos": 0.9999, "grad_rel": 1e-3}
# The two-network model on 16^3 particles: a few voxels have a ReLU pre-activation within
# ~1e-6 of zero, where the FP32 sum may take the other side of the kink than the FP64 oracle
# and that voxel's derivative changes (measured gradient rel-L2 7.8e-3 on the 32^3 meshes,
# 1.0e-3 on the 16^3 mesh; cosine 0.99997).
TOL_FP32_KINK = dict(TOL_FP32, grad_rel=1e-2)


def test_density_l2_small_box():
    """32^3 particles on a 32^3 mesh, L = 100 Mpc/h, 5 steps, density-L2 loss."""
    require_gpu()
    say("pipeline: density-L2 32^3")
    prob = _problem(32, 32, 32, 100.0, 5, OM.LOSS_DENSITY_L2, 1)
    res = _gpu_run(*prob)
    _compare(*prob, res, TOL_FP32)


def test_lognormal_batch_with_anneal_stages():
    """Two items with different residual smoothing (R_sm = 0 and 4 Mpc/h), 32^3, H = 32."""
    require_gpu()
    say("pipeline: log-normal 32^3, B=2")
    prob = _problem(32, 32, 32, 100.0, 4, OM.LOSS_LOGNORMAL, 2, hidden=32, R_sm=(0.0, 4.0))
    res = _gpu_run(*prob, hidden=32)
    _compare(*prob, res, TOL_FP32)


def test_lognormal_data_term_alone():
    """Prior weight 0: the gradient is the data term's alone (PM + network + likelihood)."""
    require_gpu()
    say("pipeline: log-normal data term only, 32^3")
    prob = _problem(32, 32, 32, 100.0, 5, OM.LOSS_LOGNORMAL, 2, hidden=32, R_sm=(2.0, 0.0),
                    prior_weight=0.0)
    res = _gpu_run(*prob, hidden=32)
    _compare(*prob, res, TOL_FP32)


def test_lognormal_mass_dependent_noise_table():
    """Per-cell mu_N, sigma_N interpolated from a table in log(M_R,data) (B = 2, R_sm = 2 and
    0); then the table switched off again gives the scalar-noise result of the same context."""
    require_gpu()
    say("pipeline: log-normal with a mass-dependent noise table, 32^3")
    prob = _problem(32, 32, 32, 100.0, 4, OM.LOSS_LOGNORMAL, 2, hidden=16, R_sm=(2.0, 0.0))
    ocfg, inv, modes, w, targets, params = prob
    lm = np.concatenate([np.log(OM.smooth(ocfg, t, params[0]["R_mass"])).ravel()
                         for t in targets])
    nodes = np.percentile(lm, [5, 35, 65, 95])
    table = (nodes, np.array([0.3, -0.1, 0.05, 0.2]), np.array([0.9, 0.35, 0.5, 0.7]))
    tparams = [dict(p, noise_table=table) for p in params]
    res = _gpu_run(ocfg, inv, modes, w, targets, tparams, hidden=16, noise=table)
    _compare(ocfg, inv, modes, w, targets, tparams, res, TOL_FP32)
    pm = res["pm"]
    pm.set_noise_table()
    m = res["modes"]
    _, loss = pm.forward(m)
    ref = _gpu_run(*prob, hidden=16)
    np.testing.assert_array_equal(loss.cpu().numpy(), ref["loss"])


def test_force_mesh_twice_particle_mesh():
    """16^3 particles, 32^3 force mesh, 16^3 output mesh, 3 steps."""
    require_gpu()
    say("pipeline: 16^3 particles on 32^3 force mesh")
    prob = _problem(16, 32, 16, 50.0, 3, OM.LOSS_LOGNORMAL, 1, hidden=8, R_sm=(1.0,))
    res = _gpu_run(*prob)
    _compare(*prob, res, TOL_FP32)


def test_checkpointing_reproduces_stored_gradient_bitwise():
    """ckpt_every = 2 recomputes steps from checkpoints; deterministic kernels make the
    gradient identical to keeping every step."""
    require_gpu()
    say("pipeline: checkpoint every 2 vs keep all")
    prob = _problem(16, 16, 16, 50.0, 5, OM.LOSS_LOGNORMAL, 2, hidden=8, R_sm=(2.0, 0.0))
    a = _gpu_run(*prob, ckpt=0)
    b = _gpu_run(*prob, ckpt=2)
    c = _gpu_run(*prob, ckpt=3)
    assert np.array_equal(a["loss"], b["loss"]) and np.array_equal(a["loss"], c["loss"])
    assert np.array_equal(a["grad"], b["grad"]), np.abs(a["grad"] - b["grad"]).max()
    assert np.array_equal(a["grad"], c["grad"])


def test_repeated_adjoint_and_recompute_guard():
    """Without recomputation a second adjoint of the same forward repeats the gradient
    bitwise; after an adjoint that recomputed checkpoint segments the per-step state of the
    last segment is gone, so another adjoint is refused until the next forward, which then
    gives the same gradient again."""
    require_gpu()
    say("pipeline: repeated adjoint, with and without recomputation")
    prob = _problem(16, 16, 16, 50.0, 5, OM.LOSS_LOGNORMAL, 1, hidden=8, R_sm=(2.0,))
    ones = torch.ones(1, dtype=torch.float64, device=DEV)
    a = _gpu_run(*prob, ckpt=0)
    assert np.array_equal(a["pm"].adjoint(ones).cpu().numpy(), a["grad"])
    b = _gpu_run(*prob, ckpt=2)
    with pytest.raises(P.PmrError):
        b["pm"].adjoint(ones)
    b["pm"].forward(b["modes"])
    assert np.array_equal(b["pm"].adjoint(ones).cpu().numpy(), b["grad"])
    assert np.array_equal(a["grad"], b["grad"])


def test_run_to_run_bitwise():
    require_gpu()
    prob = _problem(32, 32, 32, 100.0, 3, OM.LOSS_LOGNORMAL, 1, hidden=16, R_sm=(2.0,))
    a = _gpu_run(*prob, hidden=16)
    b = _gpu_run(*prob, hidden=16)
    assert np.array_equal(a["loss"], b["loss"])
    assert np.array_equal(a["grad"], b["grad"])
    assert np.array_equal(a["mass"], b["mass"])


# BF16 network with FP32 accumulation (measured: loss <= 2.9e-4, mass <= 1.8e-3, gradient
# rel-L2 <= 1.4e-3).
TOL_MIXED = {"max_dx_cells": 1e-4, "delta_f": 1e-4, "prior": 1e-5, "loss": 1e-3, "mass": 2e-2,
             "grad_cos": 0.999, "grad_rel": 3e-2}


@pytest.mark.parametrize("hidden", [32, 64])
def test_mixed_precision_network(hidden):
    """BF16 matrix-core network (FP32 accumulation) against the FP64 oracle."""
    require_gpu()
    say(f"pipeline: mixed precision, H={hidden}")
    prob = _problem(32, 32, 32, 100.0, 3, OM.LOSS_LOGNORMAL, 2, hidden=hidden, R_sm=(2.0, 0.0))
    res = _gpu_run(*prob, hidden=hidden, precision=P.PMR_MIXED)
    _compare(*prob, res, TOL_MIXED)


@pytest.fixture
def tile_shape():
    """Sets the FFT tile shape of given sizes (both strided passes) for one test and restores
    it afterwards."""
    saved = {}

    def set_shape(n, pc, nth, staging):
        for p in (P.PMR_FFT_YPASS, P.PMR_FFT_XPASS, P.PMR_FFT_XPASS_MULTI):
            if (n, p) not in saved:
                saved[(n, p)] = P.fft_get_tile(n, p)
            P.fft_set_tile(n, p, pc, nth, staging)

    yield set_shape
    for (n, p), v in saved.items():
        P.fft_set_tile(n, p, *v)


@pytest.mark.parametrize("staging", [0, 1, 2])
def test_register_and_lds_fft_staging_64_on_128(tile_shape, staging):
    """64^3 particles on a 128^3 force mesh (64^3 output), 3 steps, H = 32: sizes where the
    strided passes and every fused k-space operator run on register images (staging 0,
    8 and 16 points per thread) or on LDS-staged tiles with radix-8 (staging 1) or radix-4
    (staging 2) stages."""
    require_gpu()
    say(f"pipeline: 64^3 on 128^3, staging {staging}")
    tile_shape(64, 32, 256, staging)
    tile_shape(128, 32, 256, staging)
    prob = _problem(64, 128, 64, 200.0, 3, OM.LOSS_LOGNORMAL, 1, hidden=32, R_sm=(2.0,))
    res = _gpu_run(*prob, hidden=32)
    _compare(*prob, res, TOL_FP32)


def test_large_mesh_shape_scaled_to_64_on_128():
    """The 256^3-particle / 512^3-mesh workload scaled down to 64^3 particles on a 128^3 force
    mesh (64^3 output) at the same box (400 Mpc/h), 10 steps, 3-64-64-1 network and
    checkpointing every 2 steps: the FP32 path and the mixed path (BF16 network) against the
    oracle, and against each other."""
    require_gpu()
    say("pipeline: 64^3 on 128^3, 10 steps, H=64, FP32 and mixed")
    prob = _problem(64, 128, 64, 400.0, 10, OM.LOSS_LOGNORMAL, 1, hidden=64, R_sm=(2.0,))
    ocfg, inv, modes, w, targets, params = prob
    refs = [OM.gradient(ocfg, modes[0], inv, targets[0], params[0], w)]
    grads = {}
    for precision, tol in ((P.PMR_FP32, TOL_FP32), (P.PMR_MIXED, TOL_MIXED)):
        say(f"  precision {precision}")
        res = _gpu_run(*prob, hidden=64, ckpt=2, precision=precision)
        _compare(*prob, res, tol, refs=refs)
        grads[precision] = res["grad"][0]
    a, b = grads[P.PMR_FP32], grads[P.PMR_MIXED]
    say(f"  mixed vs FP32: grad rel-L2 {rel_l2(b, a):.3e}, cos {cosine(b, a):.6f}")


@pytest.mark.parametrize("hidden", [8, 16])
def test_small_networks(hidden):
    """H = 8 (vector units) and H = 16 (FP32 matrix cores, one 16-wide block), 16^3, 3 steps."""
    require_gpu()
    say(f"pipeline: 16^3, H={hidden}")
    prob = _problem(16, 16, 16, 50.0, 3, OM.LOSS_LOGNORMAL, 2, hidden=hidden, R_sm=(1.0, 0.0))
    res = _gpu_run(*prob, hidden=hidden)
    _compare(*prob, res, TOL_FP32)


def test_second_order_lpt_density_l2():
    """Second-order LPT initial conditions (32^3 particles, 64^3 force mesh, B = 2): the
    positions, loss and mode gradient against the oracle; the second-order displacement
    alone (x0 of the 2LPT run minus x0 of the Zel'dovich run of the same modes) against the
    oracle's (3/7) D0^2 Psi2; a second adjoint reproduces the first bit for bit."""
    require_gpu()
    say("pipeline: 2LPT density-L2 32^3 / 64^3 mesh, B=2")
    prob = _problem(32, 64, 64, 100.0, 4, OM.LOSS_DENSITY_L2, 2, ic_order=2)
    ocfg, inv, modes, w, targets, params = prob
    res = _gpu_run(*prob)
    _compare(*prob, res, TOL_FP32)
    g2 = res["pm"].adjoint(torch.ones(2, dtype=torch.float64, device=DEV)).cpu().numpy()
    assert np.array_equal(g2, res["grad"])
    c1 = OM.Config(ocfg.box, 32, 64, 64, 4, loss_kind=OM.LOSS_DENSITY_L2, ic_order=1)
    res1 = _gpu_run(c1, inv, modes, w, targets, params)
    D = ocfg.fac["D0"]
    for b in range(2):
        _, _, _, extra = OM.zeldovich(ocfg, modes[b], full=True)
        ref = OM.LPT2_D * D * D * extra["psi2"]
        d = res["xs"][0][b] - res1["xs"][0][b]
        d = (d + ocfg.box / 2) % ocfg.box - ocfg.box / 2
        e = rel_l2(d, ref)
        say(f"  item {b}: second-order displacement rel_l2={e:.3e}, "
            f"rms={np.sqrt(np.mean(ref ** 2)) / (ocfg.box / 64):.3e} cells")
        assert e < 1e-3, e


def test_second_order_lpt_lognormal_with_checkpoints():
    """2LPT with the log-normal likelihood and checkpointed steps (32^3, H = 32, 6 steps,
    a checkpoint every 2 steps)."""
    require_gpu()
    say("pipeline: 2LPT log-normal 32^3, ckpt 2")
    prob = _problem(32, 32, 32, 100.0, 6, OM.LOSS_LOGNORMAL, 1, hidden=32, R_sm=(2.0,),
                    ic_order=2)
    res = _gpu_run(*prob, hidden=32, ckpt=2)
    _compare(*prob, res, TOL_FP32)


def _two_net_problem(n, nm, box, steps, B, R_sm, a, seed=1):
    """Output mesh = force mesh (nm)."""
    ocfg = OM.Config(box, n, nm, nm, steps, loss_kind=OM.LOSS_LOGNORMAL,
                     halo_model=OM.HALO_TWO)
    power = OC.bbks_power()
    inv = OM.prior_inv_variance(n, box, power)
    nets = synth.halo_net_weights(3)
    modes, targets, params = [], [], []
    for b in range(B):
        modes.append(OM.linear_modes(synth.white_noise(seed + 10 * b, n), box, power))
        st = OM.linear_modes(synth.white_noise(seed + 10 * b + 5, n), box, power)
        t = OM.forward(ocfg, st, inv, np.ones((nm,) * 3), OM.default_params(), nets)["mass"]
        targets.append(t)
        params.append(OM.default_params(M0=float(np.percentile(t, 60)), R_sm=R_sm[b], mu=0.1,
                                        logistic_a=a[b]))
    return ocfg, inv, modes, nets, targets, params


def test_two_network_halo_model():
    """The paper's position x mass networks (32^3, B = 2 with the anneal ends a = 1, R_sm = 2
    and a = 3, R_sm = 0): mass field, loss and mode gradient against the oracle."""
    require_gpu()
    say("pipeline: two-network halo model 32^3, B=2")
    prob = _two_net_problem(32, 32, 100.0, 4, 2, (2.0, 0.0), (1.0, 3.0))
    res = _gpu_run(*prob)
    _compare(*prob, res, TOL_FP32)


def test_two_network_halo_model_on_the_force_mesh():
    """Force and output meshes at twice the particle resolution (16^3 particles, 32^3
    meshes), a = 2."""
    require_gpu()
    say("pipeline: two-network halo model 16^3 particles, 32^3 meshes")
    prob = _two_net_problem(16, 32, 60.0, 3, 1, (1.0,), (2.0,), seed=6)
    res = _gpu_run(*prob)
    _compare(*prob, res, TOL_FP32_KINK)


def test_second_order_lpt_with_two_networks_64():
    """Both next rows together at 64^3 (many 16-voxel groups per wavefront of the matrix-core
    kernels, the register-staged FFT passes), against the oracle; then the same gradient
    captured as a HIP graph and replayed (with eager work in between) reproduces the eager
    result bit for bit."""
    require_gpu()
    say("pipeline: 2LPT + two-network model 64^3, and graph replay")
    n, box = 64, 200.0
    ocfg = OM.Config(box, n, n, n, 4, loss_kind=OM.LOSS_LOGNORMAL, ic_order=2,
                     halo_model=OM.HALO_TWO)
    power = OC.bbks_power()
    inv = OM.prior_inv_variance(n, box, power)
    nets = synth.halo_net_weights(5)
    s = OM.linear_modes(synth.white_noise(31, n), box, power)
    t = OM.forward(ocfg, OM.linear_modes(synth.white_noise(32, n), box, power), inv,
                   np.ones((n,) * 3), OM.default_params(), nets)["mass"]
    prm = OM.default_params(M0=float(np.percentile(t, 60)), R_sm=2.0, mu=0.1, logistic_a=2.0)
    res = _gpu_run(ocfg, inv, [s], nets, [t], [prm])
    _compare(ocfg, inv, [s], nets, [t], [prm], res, TOL_FP32)
    pm, m = res["pm"], res["modes"]
    G = P.GradientGraph(pm, m)
    ones = torch.ones(1, dtype=torch.float64, device=DEV)
    ref_loss = torch.from_numpy(res["loss"]).to(DEV)
    ref_grad = torch.from_numpy(res["grad"]).to(DEV)
    for rep in range(3):
        G.modes.copy_(m)
        loss, grad = G.replay()
        torch.cuda.synchronize()
        assert torch.equal(loss, ref_loss), rep
        assert torch.equal(grad, ref_grad), rep
        pm.forward(m, want_mass=False)
        pm.adjoint(ones)


def test_non_finite_loss_check():
    """pmr_set_check_finite: a data field with a NaN makes the loss NaN; with the check on the
    forward reports PMR_E_NONFINITE (outputs still written, the adjoint may follow), with it
    off the forward succeeds and returns the NaN loss."""
    require_gpu()
    say("pipeline: non-finite loss check")
    prob = _problem(16, 16, 16, 60.0, 2, OM.LOSS_LOGNORMAL, 1)
    ocfg, inv, modes, w, targets, params = prob
    bad = targets[0].copy()
    bad[3, 4, 5] = np.nan
    cfg = P.Config(batch=1, n_part=16, n_mesh=16, n_out=16, n_steps=2, mlp_hidden=8, box=60.0)
    pm = P.PMContext(cfg, DEV)
    pm.set_prior(torch.from_numpy(inv.astype(np.float32)))
    pm.set_mlp({k: torch.from_numpy(v) for k, v in w.items()})
    pm.set_loss(P.LossParams(M0=params[0]["M0"], mu=params[0]["mu"]))
    m = torch.from_numpy(modes[0].astype(np.complex64)).reshape(1, -1).to(DEV)
    pm.set_target(torch.from_numpy(targets[0].astype(np.float32)).reshape(1, -1))
    pm.set_check_finite(True)
    _, loss = pm.forward(m)  # finite: no error
    assert np.isfinite(loss.cpu().numpy()).all()
    pm.set_target(torch.from_numpy(bad.astype(np.float32)).reshape(1, -1))
    with pytest.raises(P.PmrError) as e:
        pm.forward(m)
    assert e.value.status == -5
    pm.adjoint(torch.ones(1, dtype=torch.float64, device=DEV))
    pm.set_check_finite(False)
    _, loss = pm.forward(m)
    assert np.isnan(loss.cpu().numpy()[0, 0])


def test_two_network_smallest_mesh_odd_batch():
    """The two-network model on the smallest mesh (16^3, one 16-voxel group per row) with an
    odd batch of 3 items, each with its own logistic sharpness."""
    require_gpu()
    say("pipeline: two-network model 16^3, B=3")
    ocfg, inv, modes, nets, targets, params = _two_net_problem(16, 16, 50.0, 3, 3,
                                                                (0.0, 1.0, 2.0), (1.0, 2.0, 3.0))
    res = _gpu_run(ocfg, inv, modes, nets, targets, params)
    _compare(ocfg, inv, modes, nets, targets, params, res, TOL_FP32_KINK)


def test_two_network_state_and_argument_errors():
    """Weights of the other halo model are refused (PMR_E_STATE), as is a non-positive
    logistic sharpness for the two-network model (PMR_E_INVALID)."""
    require_gpu()
    nets = synth.halo_net_weights(3)
    single = P.PMContext(P.Config(batch=1, n_part=16, n_mesh=16, n_out=16, n_steps=1,
                                  mlp_hidden=8), DEV)
    with pytest.raises(P.PmrError) as e:
        single.set_halo_nets(nets)
    assert e.value.status == -6
    two = P.PMContext(P.Config(batch=1, n_part=16, n_mesh=16, n_out=16, n_steps=1,
                               halo_model=P.PMR_HALO_TWO), DEV)
    with pytest.raises(P.PmrError) as e:
        two.set_mlp({k: torch.from_numpy(v) for k, v in synth.mlp_weights(3, 32).items()})
    assert e.value.status == -6
    with pytest.raises(P.PmrError) as e:
        two.set_loss(P.LossParams(logistic_a=0.0))
    assert e.value.status == -1
    two.set_loss(P.LossParams(logistic_a=1.5))


def test_zero_modes_keep_the_lattice():
    """The degenerate input: all linear modes zero. With L = 64 on a 32^3 lattice and mesh
    (cell 2, lattice at cell centres: every CIC fraction is exactly 1/2), the painted density
    is exactly uniform, so the force is exactly zero: every position after every step equals
    the lattice bit for bit, the final density contrast is exactly 0 and so is the prior
    term. The mode gradient (the data term alone, through the whole adjoint) still has to
    match the oracle's."""
    require_gpu()
    say("pipeline: zero modes, 32^3, L = 64")
    ocfg, inv, modes, w, targets, params = _problem(32, 32, 32, 64.0, 3, OM.LOSS_LOGNORMAL, 2,
                                                    hidden=8, R_sm=(2.0, 0.0))
    modes = [np.zeros_like(m) for m in modes]
    res = _gpu_run(ocfg, inv, modes, w, targets, params)
    q = M.lattice_positions(32, 64.0, 32)
    for i, x in enumerate(res["xs"]):
        for b in range(2):
            assert np.array_equal(x[b], q), i
    assert np.all(res["delta_f"] == 0.0)
    assert np.all(res["loss"][:, 1] == 0.0)
    _compare(ocfg, inv, modes, w, targets, params, res,
             {k: v for k, v in TOL_FP32.items() if k != "delta_f"})


def test_sort_event_timing_counts_its_launches():
    """The sort timing class brackets every kernel of one cell sort as one launch: a 3-step
    forward at 32^3 runs 4 sorts (one per step, one on the output mesh); the sort is an
    implementation cost, so its algorithmic bytes are 0."""
    require_gpu()
    say("profile class sort, 32^3, 3 steps")
    ocfg, inv, modes, w, targets, params = _problem(32, 32, 32, 100.0, 3, OM.LOSS_DENSITY_L2, 1)
    res = _gpu_run(ocfg, inv, modes, w, targets, params)
    pm = res["pm"]
    pm.profile_begin("sort")
    pm.forward(res["modes"], want_mass=False)
    ms, n, nbytes = pm.profile_end()
    assert n == 4
    assert nbytes == 0.0
    assert ms > 0.0


@pytest.mark.parametrize("columns", [8, 16, 32])
def test_kz_slab_windows_equal_whole_passes(columns):
    """The force transforms of the PM steps run slab by slab of kz columns (y pass, x pass
    with the force or force-adjoint operator, inverse y pass per window): every tile is the
    same computation as in whole passes, so the gradient and loss are equal bit for bit
    (64^3 particles on a 128^3 mesh: 65 kz columns, the last window partial)."""
    require_gpu()
    say(f"pipeline: kz slabs of {columns} columns on the 128^3 force mesh")
    prob = _problem(64, 128, 64, 200.0, 3, OM.LOSS_LOGNORMAL, 1, hidden=32, R_sm=(2.0,))
    saved = P.fft_get_slab(128)
    try:
        P.fft_set_slab(128, 0)
        a = _gpu_run(*prob, hidden=32)
        P.fft_set_slab(128, columns)
        b = _gpu_run(*prob, hidden=32)
    finally:
        P.fft_set_slab(128, saved)
    assert np.array_equal(a["loss"], b["loss"])
    assert np.array_equal(a["grad"], b["grad"])
    assert np.array_equal(a["mass"], b["mass"])


@pytest.mark.parametrize("rows", [1, 2, 4, 8])
def test_paint_rows_per_wave_against_oracle(rows):
    """Every rows-per-wavefront setting of the paints (the density and the adjoint's three
    channels on the 128^3 force mesh, the final paint on the 64^3 output mesh) against the
    oracle, and bitwise reproducible for the setting."""
    require_gpu()
    say(f"pipeline: paints with {rows} rows per wavefront, 64^3 on 128^3")
    prob = _problem(64, 128, 64, 200.0, 3, OM.LOSS_LOGNORMAL, 1, hidden=32, R_sm=(2.0,))
    keys = [(128, 1), (128, 3), (64, 1)]
    saved = {k: P.paint_get_rows(*k) for k in keys}
    try:
        for k in keys:
            P.paint_set_rows(*k, rows)
        res = _gpu_run(*prob, hidden=32)
        again = _gpu_run(*prob, hidden=32)
    finally:
        for k, v in saved.items():
            P.paint_set_rows(*k, v)
    _compare(*prob, res, TOL_FP32)
    assert np.array_equal(res["grad"], again["grad"]) and np.array_equal(res["loss"], again["loss"])


@pytest.mark.parametrize("ckpt", [1, 2, 3])
def test_checkpointed_positions_equal_stored(ckpt):
    """With checkpointing the positions at segment starts live in the checkpoints (written
    by the steps before them) and the last segment in ring slots: every position the
    context holds after a forward equals the one of the run that keeps every step, bit for
    bit, and positions the ring no longer holds are refused (PMR_E_STATE)."""
    require_gpu()
    say(f"pipeline: positions held with checkpoints every {ckpt} steps, 32^3, 7 steps")
    prob = _problem(32, 32, 32, 100.0, 7, OM.LOSS_LOGNORMAL, 2, hidden=16, R_sm=(0.0, 2.0))
    ref = _gpu_run(*prob, hidden=16)
    res = _gpu_run(*prob, hidden=16, ckpt=ckpt)
    assert np.array_equal(res["grad"], ref["grad"]) and np.array_equal(res["loss"], ref["loss"])
    pm = res["pm"]
    pm.forward(res["modes"], want_mass=False)
    n = 7
    lo = ((n - 1) // ckpt) * ckpt
    for step in range(n + 1):
        if step % ckpt == 0 or step >= lo:
            assert np.array_equal(pm.debug("x", step).cpu().numpy(), ref["xs"][step]), step
        else:
            with pytest.raises(P.PmrError) as e:
                pm.debug("x", step)
            assert e.value.status == P.PMR_E_STATE


@pytest.mark.parametrize("n,nm", [(16, 16), (16, 32), (32, 32)])
def test_force_meshes_every_step_against_oracle(n, nm):
    """The force mesh of every PM step (the operator split over the axes: i k_x / k^2 in the
    x pass, i k_y and i k_z of the potential in the y pass) against the FP64 oracle's
    irfft(i k_a / k^2 rfft(delta)) from the GPU's own positions, component by component, on
    meshes small enough that the Nyquist planes and k = 0 carry a visible share of the
    spectrum; the later steps paint clustered positions."""
    require_gpu()
    say(f"pipeline: force meshes of every step, {n}^3 particles on {nm}^3")
    steps = 4
    prob = _problem(n, nm, n, 50.0, steps, OM.LOSS_LOGNORMAL, 2, hidden=8, R_sm=(1.0,))
    res = _gpu_run(*prob)
    ocfg = prob[0]
    worst = 0.0
    for i in range(steps):
        F = res["pm"].debug("force", i).cpu().numpy()  # [B][nm^3][3]
        for b in range(2):
            ref = OM.force_meshes(ocfg, OM.density(ocfg, res["xs"][i][b].astype(np.float64), nm))
            for a in range(3):
                e = rel_l2(F[b][:, a], ref[a].ravel())
                worst = max(worst, e)
                assert e <= 2e-6, (i, b, "xyz"[a], e)  # measured 2.4-2.8e-7
    say(f"  worst component rel-L2 {worst:.2e}")
