"""A gradient evaluation captured as a HIP graph replays bit-identically to eager calls,
including across eager work in between replays and after a change of loss parameters."""
import numpy as np
import pytest
import torch

import synth
from oracle import cosmology as OC
from oracle import model as OM
import paper_1805_02247_amd as P
from _gpu import DEV, require_gpu, say

pytestmark = pytest.mark.gpu


def test_graph_replay_matches_eager():
    require_gpu()
    n, box, B = 32, 100.0, 2
    say("graph: capture one gradient evaluation, replay 4 times")
    power = OC.bbks_power()
    inv = OM.prior_inv_variance(n, box, power)
    w = synth.mlp_weights(3, 16)
    cfg = P.Config(batch=B, n_part=n, n_mesh=n, n_out=n, n_steps=3, mlp_hidden=16, box=box,
                   ckpt_every=2)
    pm = P.PMContext(cfg, DEV)
    pm.set_prior(torch.from_numpy(inv.astype(np.float32)))
    pm.set_mlp({k: torch.from_numpy(v) for k, v in w.items()})
    tgt = np.stack([np.exp(synth.unit_normal(40 + b, (n, n, n))) for b in range(B)])
    pm.set_target(torch.from_numpy(tgt.astype(np.float32)).reshape(B, -1))
    params = [P.LossParams(M0=1.0, R_sm=2.0), P.LossParams(M0=1.5, R_sm=0.0)]
    pm.set_loss(params)
    modes = [torch.from_numpy(OM.linear_modes(synth.white_noise(s, n), box, power)
                              .astype(np.complex64).reshape(-1)) for s in (1, 2)]
    m0 = torch.stack(modes).to(DEV)
    m1 = torch.stack(modes[::-1]).to(DEV)

    def eager(m):
        _, loss = pm.forward(m, want_mass=False)
        g = pm.adjoint(torch.ones(B, dtype=torch.float64, device=DEV))
        torch.cuda.synchronize()
        return loss.clone(), g.clone()

    ref0 = eager(m0)
    ref1 = eager(m1)
    G = P.GradientGraph(pm, m0)
    for rep in range(4):
        m = m0 if rep % 2 == 0 else m1
        ref = ref0 if rep % 2 == 0 else ref1
        G.modes.copy_(m)
        loss, grad = G.replay()
        torch.cuda.synchronize()
        assert torch.equal(loss, ref[0]), rep
        assert torch.equal(grad, ref[1]), rep
        eager(m1)  # eager work between replays
    # new anneal stage (R_sm and M0 change): replay right after set_loss, then compare
    # with the eager evaluation at the same parameters
    new = [P.LossParams(M0=1.2, R_sm=4.0), P.LossParams(M0=2.0, R_sm=1.0)]
    pm.set_loss(new)
    G.modes.copy_(m0)
    loss, grad = G.replay()
    torch.cuda.synchronize()
    loss, grad = loss.clone(), grad.clone()
    ref2 = eager(m0)
    assert torch.equal(loss, ref2[0]) and torch.equal(grad, ref2[1])
    assert not torch.equal(ref2[0], ref0[0])


@pytest.mark.parametrize("capture", [True, False])
def test_graph_with_device_loss_params(capture):
    """Loss parameters from device memory, read by pmr_set_loss_device inside the graph
    (capture) or applied on the stream when they change: new anneal-stage values written
    into the device buffer between replays give, bit for bit, the eager gradient at those
    values (set through the host call), without recapture; an invalid item (sigma_N = 0)
    gives a NaN loss for that item only."""
    require_gpu()
    n, box, B = 32, 100.0, 2
    say("graph: device loss parameters, stage changes between replays")
    power = OC.bbks_power()
    inv = OM.prior_inv_variance(n, box, power)
    w = synth.mlp_weights(3, 16)
    cfg = P.Config(batch=B, n_part=n, n_mesh=n, n_out=n, n_steps=3, mlp_hidden=16, box=box)
    pm = P.PMContext(cfg, DEV)
    pm.set_prior(torch.from_numpy(inv.astype(np.float32)))
    pm.set_mlp({k: torch.from_numpy(v) for k, v in w.items()})
    tgt = np.stack([np.exp(synth.unit_normal(50 + b, (n, n, n))) for b in range(B)])
    pm.set_target(torch.from_numpy(tgt.astype(np.float32)).reshape(B, -1))
    stages = [[P.LossParams(M0=1.0, R_sm=4.0), P.LossParams(M0=1.5, R_sm=2.0)],
              [P.LossParams(M0=0.8, R_sm=1.0), P.LossParams(M0=1.1, R_sm=0.0)],
              [P.LossParams(M0=1.3, R_sm=0.0, R_mass=2.0), P.LossParams(M0=0.7, R_sm=1.0)]]
    pm.set_loss(stages[0])
    m = torch.from_numpy(OM.linear_modes(synth.white_noise(3, n), box, power)
                         .astype(np.complex64).reshape(1, -1)).repeat(B, 1).to(DEV)

    def eager(prm):
        pm.set_loss(prm)
        _, loss = pm.forward(m, want_mass=False)
        g = pm.adjoint(torch.ones(B, dtype=torch.float64, device=DEV))
        torch.cuda.synchronize()
        return loss.clone(), g.clone()

    refs = [eager(st) for st in stages]
    G = P.GradientGraph(pm, m, params=stages[0], capture_params=capture)
    for rep, k in enumerate((0, 1, 2, 1, 0)):
        G.set_params(stages[k])
        loss, grad = G.replay()
        torch.cuda.synchronize()
        assert torch.equal(loss, refs[k][0]), (rep, k)
        assert torch.equal(grad, refs[k][1]), (rep, k)
        eager(stages[(k + 1) % 3])  # eager work (other parameters) between replays
    bad = [P.LossParams(M0=1.0, R_sm=4.0, sigma_N=0.0), stages[0][1]]
    G.set_params(bad)
    loss, _ = G.replay()
    torch.cuda.synchronize()
    lv = loss.cpu().numpy()
    assert np.all(np.isnan(lv[0])) and np.all(np.isfinite(lv[1]))
    assert np.array_equal(lv[1], refs[0][0].cpu().numpy()[1])
