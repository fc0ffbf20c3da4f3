"""PMForward, the torch.autograd.Function over pmr_forward / pmr_adjoint: loss.backward()
gives the hand-written adjoint's gradient for flat and 4-D mode tensors, with and without a
mass cotangent, matches the FP64 oracle, and a backward after a later forward on the same
context is refused (PMR_E_STATE) instead of returning the later forward's gradient."""
import numpy as np
import pytest
import torch

import synth
from oracle import cosmology as OC
from oracle import model as OM
import paper_1805_02247_amd as P
from _gpu import DEV, cosine, rel_l2, require_gpu, say

pytestmark = pytest.mark.gpu

N, BOX, STEPS, B, H = 32, 100.0, 3, 2, 16


def _setup():
    power = OC.bbks_power()
    inv = OM.prior_inv_variance(N, BOX, power)
    w = synth.mlp_weights(3, H)
    ocfg = OM.Config(BOX, N, N, N, STEPS)
    targets = [np.exp(0.5 * synth.unit_normal(60 + b, (N, N, N))) for b in range(B)]
    params = [OM.default_params(M0=float(np.median(targets[b])), R_sm=(2.0, 0.0)[b], mu=0.1)
              for b in range(B)]
    modes = [OM.linear_modes(synth.white_noise(70 + b, N), BOX, power) for b in range(B)]
    cfg = P.Config(batch=B, n_part=N, n_mesh=N, n_out=N, n_steps=STEPS, mlp_hidden=H, box=BOX)
    pm = P.PMContext(cfg, DEV)
    pm.set_prior(torch.from_numpy(inv.astype(np.float32)))
    pm.set_mlp({k: torch.from_numpy(v) for k, v in w.items()})
    pm.set_target(torch.from_numpy(np.stack(targets).astype(np.float32)).reshape(B, -1))
    pm.set_loss([P.LossParams(**p) for p in params])
    m = torch.from_numpy(np.stack(modes).astype(np.complex64)).reshape(B, -1).to(DEV)
    return pm, m, (ocfg, inv, w, targets, params)


def _adjoint(pm, m, loss_bar, mass_bar=None):
    pm.forward(m)
    g = pm.adjoint(loss_bar, mass_bar)
    torch.cuda.synchronize()
    return g


def test_backward_equals_adjoint_and_oracle():
    require_gpu()
    say("autograd: PMForward on flat modes vs pmr_adjoint and the oracle")
    pm, m, (ocfg, inv, w, targets, params) = _setup()
    x = m.clone().requires_grad_(True)
    loss, mass = P.PMForward.apply(x, pm)
    assert loss.shape == (B,) and mass.shape == (B, N ** 3)
    loss.sum().backward()
    assert x.grad.shape == m.shape
    ref = _adjoint(pm, m, torch.ones(B, dtype=torch.float64, device=DEV))
    assert torch.equal(x.grad, ref)
    for b in range(B):
        s = m[b].cpu().numpy().astype(np.complex128).reshape(N, N, N // 2 + 1)
        _, G = OM.gradient(ocfg, s, inv, targets[b], params[b], w)
        g = x.grad[b].cpu().numpy().reshape(G.shape)
        say(f"  item {b}: grad rel-L2 {rel_l2(g, G):.2e}, cos {cosine(g, G):.8f}")
        assert cosine(g, G) >= 0.9999 and rel_l2(g, G) <= 1e-3


def test_backward_four_dimensional_modes_and_mass_cotangent():
    require_gpu()
    say("autograd: 4-D modes, loss weights and a mass cotangent")
    pm, m, _ = _setup()
    m4 = m.reshape(B, N, N, N // 2 + 1)
    x = m4.clone().requires_grad_(True)
    loss, mass = P.PMForward.apply(x, pm)
    wl = torch.tensor([0.5, 2.0], dtype=torch.float64, device=DEV)
    wm = torch.from_numpy(synth.unit_normal(80, (B, N ** 3)).astype(np.float32)).to(DEV)
    ((loss * wl).sum() + (mass * wm).sum()).backward()
    assert x.grad.shape == m4.shape
    ref = _adjoint(pm, m, wl, wm)
    assert torch.equal(x.grad.reshape(B, -1), ref)


def test_stale_backward_is_refused():
    require_gpu()
    say("autograd: a backward after a later forward on the same context")
    pm, m, _ = _setup()
    x = m.clone().requires_grad_(True)
    loss1, _ = P.PMForward.apply(x, pm)
    loss2, _ = P.PMForward.apply(x * 0.5, pm)
    with pytest.raises(P.PmrError) as e:
        loss1.sum().backward()
    assert e.value.status == P.PMR_E_STATE
    x.grad = None
    loss2.sum().backward()  # the latest forward still differentiates
    assert x.grad is not None and torch.isfinite(torch.view_as_real(x.grad)).all()
