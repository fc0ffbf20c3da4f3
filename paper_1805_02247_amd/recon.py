"""Reconstruction driver (Sec. 5.2, Sec. 5.3): L-BFGS over the linear modes of one
realisation, run over an anneal schedule of loss stages, and the binned two-point
statistics of Sec. 4.3 that score the result against the true modes.

Every vector operation runs in libpmr kernels: FP64 inner products with device-resident
scalars, the two-loop recursion (pmr_lbfgs_direction) and the updates; an evaluation can be
one HIP-graph replay of forward + adjoint (GradientGraph with device loss parameters).
Two drivers share the rules below. `minimize` keeps the control flow on the host: the
Armijo test on the loss copied back once per evaluation, the curvature test on three inner
products copied back once per accepted step, the history ring and the stopping rule.
`DeviceLBFGS` moves all of it to the device (pmr_lbfgs_init/trial/update): one captured
graph per evaluation holds the trial point, forward, adjoint, the Armijo and curvature tests,
the history update and the next direction, and the host only reads the status block every
few replays. On the same losses and inner products both take the same decisions and
iterates, bit for bit (the scalar tests are the same FP64 expressions, rounded once per
operation in the same order). The parameters are all stored real and imaginary parts of
the modes, so the complex64 mode tensor is used as a float32 vector of twice its length.

Readings (the paper names L-BFGS and the anneal but gives no optimiser parameters):
history m = 10; the first iteration of a stage moves a unit distance along -g (step
1 / |g|), later ones start the backtracking at step 1; Armijo constant c1 = 1e-4, at most
30 halvings (failure ends the stage); a pair is kept only if s.y > 1e-10 |s| |y|; a
non-descent direction clears the history; a stage ends when the loss falls by less than
0.1% of its value between successive iterations (Sec. 5.3), at a zero gradient, or after
max_iter iterations (the rule is not applied to a unit-length step taken without history);
each stage starts from the previous optimum with an empty history.
"""
import ctypes
import math
import time
from dataclasses import dataclass, field

import torch

from . import _lib as L
from .api import GradientGraph, LossParams, _ptr, _stream

HISTORY = 10
C1 = 1e-4
MAX_HALVINGS = 30
CURVATURE_EPS = 1e-10
REL_TOL = 1e-3


class VecOps:
    """FP64 inner products, updates and L-BFGS directions on float32 device vectors of n."""

    def __init__(self, n, m, device):
        self.n, self.m = int(n), int(m)
        nb = int(L.lib().pmr_vec_work_bytes(self.n, self.m))
        self.work = torch.empty(nb // 8 + 1, dtype=torch.float64, device=device)

    def dot(self, a, b, out):
        """out: a 0-d or 1-element float64 device tensor view."""
        L.check(L.lib().pmr_vec_dot(self.n, _ptr(a), _ptr(b), _ptr(out), _ptr(self.work),
                                    _stream()))

    def axpby(self, alpha, a, beta, b, out):
        L.check(L.lib().pmr_vec_axpby(self.n, float(alpha), _ptr(a), float(beta), _ptr(b),
                                      _ptr(out), _stream()))

    def direction(self, g, d, order, S, Y, sy, yy):
        cnt = len(order)
        arr = (ctypes.c_int * max(cnt, 1))(*order)
        L.check(L.lib().pmr_lbfgs_direction(self.n, self.m, cnt, arr, _ptr(S), _ptr(Y), _ptr(sy),
                                            _ptr(yy), _ptr(g), _ptr(d), _ptr(self.work),
                                            _stream()))


def _floats(modes):
    return modes.view(torch.float32).reshape(-1)


@dataclass
class StageResult:
    params: LossParams
    losses: list = field(default_factory=list)
    times: list = field(default_factory=list)  # wall time (s from the stage start) per loss
    evals: int = 0
    iters: int = 0
    reason: str = "max_iter"
    seconds: float = 0.0
    replays: int = 0  # graph replays (device driver: including those after the stage ended)


def minimize(pm, modes, max_iter=100, m=HISTORY, rel_tol=REL_TOL, log=None, stop_below=None,
             graph=None, c1=C1, max_halvings=MAX_HALVINGS):
    """L-BFGS from `modes` (complex64 [1][n_modes], updated in place) with the loss already
    set on `pm` (a PMContext of batch 1), or on `graph` (an api.GradientGraph of pm captured
    with device loss parameters, whose replays then evaluate forward + adjoint as one graph
    launch). stop_below: optional loss at which to stop early. Returns a StageResult."""
    if pm.cfg.batch != 1:
        raise ValueError("the driver optimises one realisation (batch 1)")
    dev = modes.device
    x = _floats(modes)
    n = x.numel()
    slots = m + 1  # the history plus one slot for the candidate pair
    ops = VecOps(n, slots, dev)
    g = torch.empty_like(x)
    xt = torch.empty_like(x)
    gt = torch.empty_like(x)
    d = torch.empty_like(x)
    S = torch.empty(slots, n, dtype=torch.float32, device=dev)
    Y = torch.empty(slots, n, dtype=torch.float32, device=dev)
    sy = torch.zeros(slots, dtype=torch.float64, device=dev)
    yy = torch.zeros(slots, dtype=torch.float64, device=dev)
    tmp = torch.zeros(4, dtype=torch.float64, device=dev)
    ones = torch.ones(1, dtype=torch.float64, device=dev)
    res = StageResult(params=None)
    t0 = time.perf_counter()

    def evaluate(src, grad_out):
        res.evals += 1
        if graph is not None:
            graph.modes.view(torch.float32).reshape(-1).copy_(src)
            loss, grad = graph.replay()
            grad_out.copy_(grad.view(torch.float32).reshape(-1))
            return float(loss[0, 0].item())
        _, loss = pm.forward(src.view(torch.complex64).reshape(1, -1), want_mass=False)
        pm.adjoint(ones, out=grad_out.view(torch.complex64).reshape(1, -1))
        return float(loss[0, 0].item())

    f = evaluate(x, g)
    res.losses.append(f)
    res.times.append(time.perf_counter() - t0)
    order = []  # history slots, newest first (at most m)
    for it in range(max_iter):
        ops.dot(g, g, tmp[0:1])
        gg = float(tmp[0].item())
        if gg == 0.0:
            res.reason = "stationary"
            break
        ops.direction(g, d, order, S, Y, sy, yy)
        ops.dot(g, d, tmp[1:2])
        gd = float(tmp[1].item())
        if gd >= 0.0:
            order = []
            ops.axpby(-1.0, g, 0.0, g, d)
            gd = -gg
        probe = not order  # unit-length step without history
        t = 1.0 if order else 1.0 / math.sqrt(gg)
        ok = False
        for _ in range(max_halvings + 1):
            ops.axpby(1.0, x, t, d, xt)
            fn = evaluate(xt, gt)
            if fn <= f + c1 * t * gd:
                ok = True
                break
            t *= 0.5
        if not ok:
            res.reason = "line_search"
            break
        slot = next(k for k in range(slots) if k not in order)
        ops.axpby(1.0, xt, -1.0, x, S[slot])
        ops.axpby(1.0, gt, -1.0, g, Y[slot])
        ops.dot(S[slot], Y[slot], sy[slot:slot + 1])
        ops.dot(Y[slot], Y[slot], yy[slot:slot + 1])
        ops.dot(S[slot], S[slot], tmp[2:3])
        h = torch.stack([sy[slot], yy[slot], tmp[2]]).cpu()
        if float(h[0]) > CURVATURE_EPS * math.sqrt(float(h[1]) * float(h[2])):
            order = ([slot] + order)[:m]  # the oldest pair leaves when m are held
        ops.axpby(1.0, xt, 0.0, xt, x)
        ops.axpby(1.0, gt, 0.0, gt, g)
        rel = (f - fn) / abs(f) if f != 0.0 else 0.0
        f = fn
        res.losses.append(f)
        res.times.append(time.perf_counter() - t0)
        res.iters = it + 1
        if log:
            log(it, f, t, res.evals)
        if stop_below is not None and f <= stop_below:
            res.reason = "target_loss"
            break
        if rel < rel_tol and not probe:
            res.reason = "converged"
            break
    torch.cuda.synchronize(dev)
    res.seconds = time.perf_counter() - t0
    return res


class _IterationGraph(GradientGraph):
    """One optimiser evaluation as a captured graph: trial point x + t d into the graph's
    modes, forward, adjoint, then the device-side test and update (pmr_lbfgs_update)."""

    def __init__(self, opt, pm, modes, params):
        self.opt = opt
        super().__init__(pm, modes, warmup=1, params=params)

    def _enqueue(self):
        o = self.opt
        xt = self.modes.view(torch.float32).reshape(-1)
        gt = self.grad.view(torch.float32).reshape(-1)
        L.check(L.lib().pmr_lbfgs_trial(o.n, _ptr(o.state), _ptr(o.x), _ptr(o.d), _ptr(xt),
                                        _stream()))
        super()._enqueue()
        L.check(L.lib().pmr_lbfgs_update(o.n, o.m, _ptr(o.state), _ptr(self.loss), _ptr(o.x),
                                         _ptr(o.g), _ptr(xt), _ptr(gt), _ptr(o.d), _ptr(o.S),
                                         _ptr(o.Y), _ptr(o.sy), _ptr(o.yy), _ptr(o.work),
                                         _stream()))


class DeviceLBFGS:
    """L-BFGS with its line search on the device (the rules of `minimize`): every
    evaluation is one replay of a graph holding the trial point, forward, adjoint, the
    Armijo test, the candidate pair with its curvature test, the move and the next
    direction, so no evaluation waits for the host. The host reads the status block every
    `check_every` replays; the replays after a stage has ended (at most check_every - 1)
    run forward + adjoint and change nothing.

    pm: a PMContext of batch 1; modes: complex64 [1][n_modes] start (the graph's shape);
    params: the first stage's LossParams (later stages: `stage(params)`)."""

    def __init__(self, pm, modes, params, m=HISTORY, max_iter=100, check_every=4):
        if pm.cfg.batch != 1:
            raise ValueError("the driver optimises one realisation (batch 1)")
        if not 1 <= m <= L.PMR_LBFGS_MAX_M:
            raise ValueError(f"history m must be in 1..{L.PMR_LBFGS_MAX_M}")
        dev = modes.device
        self.pm, self.m, self.max_iter, self.check_every = pm, int(m), int(max_iter), int(check_every)
        self.n = 2 * pm.n_modes
        f32 = dict(dtype=torch.float32, device=dev)
        self.x = torch.empty(self.n, **f32)
        self.g = torch.empty(self.n, **f32)
        self.d = torch.empty(self.n, **f32)
        self.S = torch.empty(m + 1, self.n, **f32)
        self.Y = torch.empty(m + 1, self.n, **f32)
        self.sy = torch.zeros(m + 1, dtype=torch.float64, device=dev)
        self.yy = torch.zeros(m + 1, dtype=torch.float64, device=dev)
        nb = int(L.lib().pmr_vec_work_bytes(self.n, 0))
        self.work = torch.empty(nb // 8 + 1, dtype=torch.float64, device=dev)
        sb = int(L.lib().pmr_lbfgs_state_bytes(self.max_iter))
        self.state = torch.zeros(sb // 8 + 1, dtype=torch.float64, device=dev)  # idle
        self.head = ctypes.sizeof(L.PmrLbfgsState)
        self.graph = _IterationGraph(self, pm, modes.reshape(1, -1), params)

    def read_state(self):
        """The status block (one device-to-host copy, synchronising)."""
        raw = self.state.view(torch.uint8)[:self.head].cpu().numpy().tobytes()
        return L.PmrLbfgsState.from_buffer_copy(raw)

    def stage(self, modes, params, rel_tol=REL_TOL, stop_below=None, c1=C1,
              max_halvings=MAX_HALVINGS):
        """One anneal stage from `modes` (complex64 [1][n_modes], updated in place) at loss
        parameters `params`. Returns a StageResult."""
        G = self.graph
        G.set_params(params)
        self.state.zero_()  # idle: the next replay only evaluates at x
        self.x.copy_(_floats(modes))
        G.modes.view(torch.float32).reshape(-1).copy_(self.x)
        res = StageResult(params=params)
        t0 = time.perf_counter()
        G.replay()
        self.g.copy_(G.grad.view(torch.float32).reshape(-1))
        p = L.PmrLbfgsParams(m=self.m, max_iter=self.max_iter, max_halvings=int(max_halvings),
                             c1=float(c1), curvature_eps=CURVATURE_EPS, rel_tol=float(rel_tol),
                             stop_below=-math.inf if stop_below is None else float(stop_below))
        L.check(L.lib().pmr_lbfgs_init(self.n, ctypes.byref(p), _ptr(self.state),
                                       _ptr(G.loss), _ptr(self.g), _ptr(self.d), _ptr(self.S),
                                       _ptr(self.Y), _ptr(self.sy), _ptr(self.yy),
                                       _ptr(self.work), _stream()))
        torch.cuda.synchronize(modes.device)
        t_init = time.perf_counter() - t0
        replays = 1
        while True:
            for _ in range(self.check_every):
                G.replay()
            replays += self.check_every
            st = self.read_state()
            if st.status != 1:
                break
        res.seconds = time.perf_counter() - t0
        hist = self.state.view(torch.uint8)[self.head:].view(torch.float64)
        k = self.max_iter + 1
        f_hist = hist[:k].cpu().numpy()
        clk = hist[k:2 * k].view(torch.int64).cpu().numpy()
        res.iters, res.evals = st.iters, st.evals
        res.reason = L.PMR_LBFGS_STATUS[st.status]
        res.losses = [float(v) for v in f_hist[:st.iters + 1]]
        res.times = [t_init + float(c - clk[0]) / (st.clock_khz * 1e3)
                     for c in clk[:st.iters + 1]]
        res.replays = replays
        _floats(modes).copy_(self.x)
        return res


def reconstruct(pm, modes, stages, max_iter=100, log=None, graph=None, stop_below=None,
                device=None):
    """Runs minimize over the anneal stages (LossParams each) in order, from `modes`
    (updated in place); with `graph` (a GradientGraph of pm captured with device loss
    parameters) each stage's parameters are written into the graph's parameter buffer and
    every evaluation is a graph replay; with `device` (a DeviceLBFGS of pm) every stage runs
    with the line search on the device (its own max_iter applies). stop_below applies to the
    last stage. Returns the list of StageResult."""
    out = []
    for i, p in enumerate(stages):
        last = i == len(stages) - 1
        if device is not None:
            out.append(device.stage(modes, p, stop_below=stop_below if last else None))
            continue
        if graph is not None:
            graph.set_params(p)
        else:
            pm.set_loss(p)
        r = minimize(pm, modes, max_iter=max_iter, log=log, graph=graph,
                     stop_below=stop_below if last else None)
        r.params = p
        out.append(r)
    return out


def power_bins(a, b, n, box, nbins):
    """Binned (count, P_aa, P_bb, P_ab) of two half spectra (complex64, n x n x (n/2+1)
    elements each, on the device) -> float64 device tensor [4][nbins]."""
    a = a.reshape(n, n, n // 2 + 1).contiguous()
    b = b.reshape(n, n, n // 2 + 1).contiguous()
    out = torch.empty(4, nbins, dtype=torch.float64, device=a.device)
    wb = int(L.lib().pmr_power_work_bytes(nbins))
    work = torch.empty(wb // 8 + 1, dtype=torch.float64, device=a.device)
    L.check(L.lib().pmr_power_bins(n, float(box), _ptr(a), _ptr(b), nbins, _ptr(out), _ptr(work),
                                   work.numel() * 8, _stream()))
    return out


def metrics(bins):
    """(r_c, stochasticity, TF) per shell from power_bins output (host float64 tensors)."""
    b = bins.cpu()
    paa, pbb, pab = b[1], b[2], b[3]
    ok = (paa * pbb) > 0
    rc = torch.where(ok, pab / torch.sqrt(torch.where(ok, paa * pbb, torch.ones_like(paa))),
                     torch.zeros_like(paa))
    tf = torch.where(paa > 0, torch.sqrt(torch.where(paa > 0, pbb / torch.where(paa > 0, paa,
                     torch.ones_like(paa)), torch.zeros_like(paa))), torch.zeros_like(paa))
    return rc, paa * (1.0 - rc ** 2), tf
