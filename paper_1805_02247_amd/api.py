"""Python binding of libpmr: device memory and streams from PyTorch, compute in HIP.

Every call forwards to the C ABI of include/pmr.h with the tensors' device pointers and
torch's current stream; nothing here computes any step of the forward model or gradient.
"""
import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib as L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, numel, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")


@dataclass
class Config:
    batch: int = 1
    n_part: int = 32
    n_mesh: int = 32
    n_out: int = 32
    n_steps: int = 5
    mlp_hidden: int = 32
    precision: int = L.PMR_FP32
    ckpt_every: int = 0
    loss_kind: int = L.PMR_LOSS_LOGNORMAL
    box: float = 100.0
    a0: float = 0.1
    a1: float = 1.0
    omega_m: float = 0.3175
    R1: float = 1.0
    R2: float = 2.0
    ic_order: int = 1  # 1: Zel'dovich initial conditions, 2: second-order LPT
    halo_model: int = L.PMR_HALO_SINGLE  # or PMR_HALO_TWO: the position x mass networks

    def c(self):
        return L.PmrConfig(self.batch, self.n_part, self.n_mesh, self.n_out, self.n_steps,
                           self.mlp_hidden, self.precision, self.ckpt_every, self.loss_kind,
                           self.box, self.a0, self.a1, self.omega_m, self.R1, self.R2,
                           self.ic_order, self.halo_model)


@dataclass
class LossParams:
    M0: float = 1.0
    mu: float = 0.0
    sigma_N: float = 0.5
    R_mass: float = 3.0
    R_sm: float = 0.0
    prior_weight: float = 1.0
    logistic_a: float = 3.0  # sharpness of the position network's logistic (two-network model)


LOSS_FIELDS = ("M0", "mu", "sigma_N", "R_mass", "R_sm", "prior_weight", "logistic_a")


def loss_param_rows(params, batch):
    """[batch] rows of the seven loss-parameter values from one LossParams or a list."""
    if isinstance(params, LossParams):
        params = [params] * batch
    if len(params) != batch:
        raise ValueError("one LossParams per batch item")
    return [tuple(float(getattr(p, k)) for k in LOSS_FIELDS) for p in params]


def workspace_bytes(cfg):
    c = cfg.c()
    return int(L.lib().pmr_workspace_bytes(ctypes.byref(c)))


class PMContext:
    """One configuration on one device: owns the workspace tensor and the library context."""

    def __init__(self, cfg, device="cuda:0"):
        self.cfg = cfg
        self.device = torch.device(device)
        nbytes = workspace_bytes(cfg)
        if nbytes == 0:
            raise L.PmrError(f"invalid configuration {cfg}")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self._ctx = ctypes.c_void_p()
        c = cfg.c()
        L.check(L.lib().pmr_create(ctypes.byref(c), ctypes.c_void_p(self._ws_ptr), nbytes,
                                   _stream(), ctypes.byref(self._ctx)))
        B, np_, no = cfg.batch, cfg.n_part, cfg.n_out
        self.n_modes = np_ * np_ * (np_ // 2 + 1)
        self.n_out3 = no ** 3

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                L.lib().pmr_destroy(ctx)
            except Exception:
                pass
            self._ctx = None

    def _sync_stream(self):
        L.check(L.lib().pmr_set_stream(self._ctx, _stream()))

    def set_prior(self, inv_var):
        inv_var = inv_var.to(self.device, torch.float32).contiguous()
        _need(inv_var, torch.float32, self.n_modes, "inv_var")
        self._sync_stream()
        L.check(L.lib().pmr_set_prior(self._ctx, _ptr(inv_var)))
        self._keep_prior = inv_var

    def set_mlp(self, w):
        H = self.cfg.mlp_hidden
        ts = []
        for k, n in (("W1", 3 * H), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H), ("b3", 1)):
            t = torch.as_tensor(w[k]).to(self.device, torch.float32).contiguous().reshape(-1)
            _need(t, torch.float32, n, k)
            ts.append(t)
        self._sync_stream()
        L.check(L.lib().pmr_set_mlp(self._ctx, *[_ptr(t) for t in ts]))
        self._keep_mlp = ts

    def set_check_finite(self, on=True):
        """With on, forward() synchronises and raises PmrError (status PMR_E_NONFINITE) when
        a loss value is NaN or infinite; the outputs are still written."""
        L.check(L.lib().pmr_set_check_finite(self._ctx, int(bool(on))))

    def set_halo_nets(self, nets):
        """Weights of the two-network model: nets = {"nnp": {W1, b1, W2, b2, W3, b3},
        "nnm": {...}} with the shapes of pmr_set_halo_nets."""
        sizes = {"nnp": ((50, 81), 50, (30, 50), 30, (1, 30), 1),
                 "nnm": ((20, 3), 20, (10, 20), 10, (1, 10), 1)}
        packed = []
        for net in ("nnp", "nnm"):
            parts = []
            for k, shape in zip(("W1", "b1", "W2", "b2", "W3", "b3"), sizes[net]):
                t = torch.as_tensor(nets[net][k]).to(torch.float32).reshape(-1)
                n = shape[0] * shape[1] if isinstance(shape, tuple) else shape
                if t.numel() != n:
                    raise ValueError(f"{net}.{k}: {t.numel()} values, expected {n}")
                parts.append(t)
            packed.append(torch.cat(parts).to(self.device).contiguous())
        _need(packed[0], torch.float32, L.PMR_NNP_FLOATS, "nnp")
        _need(packed[1], torch.float32, L.PMR_NNM_FLOATS, "nnm")
        self._sync_stream()
        L.check(L.lib().pmr_set_halo_nets(self._ctx, _ptr(packed[0]), _ptr(packed[1])))
        self._keep_mlp = packed

    def set_target(self, target):
        target = target.to(self.device, torch.float32).contiguous()
        _need(target, torch.float32, self.cfg.batch * self.n_out3, "target")
        self._sync_stream()
        L.check(L.lib().pmr_set_target(self._ctx, _ptr(target)))
        self._keep_target = target

    def set_loss(self, params):
        arr = (L.PmrLossParams * self.cfg.batch)(*[L.PmrLossParams(*v)
                                                    for v in loss_param_rows(params, self.cfg.batch)])
        self._sync_stream()
        L.check(L.lib().pmr_set_loss(self._ctx, arr))

    def set_loss_device(self, params):
        """Loss parameters from a device float64 tensor [B][7] (the fields of LossParams in
        order), read by the stream when it reaches this call; invalid items give a NaN loss."""
        _need(params, torch.float64, self.cfg.batch * 7, "params")
        self._sync_stream()
        L.check(L.lib().pmr_set_loss_device(self._ctx, _ptr(params)))

    def forward_count(self):
        """Number of forward passes enqueued on this context."""
        return int(L.lib().pmr_forward_count(self._ctx))

    def set_noise_table(self, log_mass=(), mu=(), sigma=()):
        """Mass-dependent noise: nodes in log(M_R,data) with mu_N and sigma_N (empty: the
        scalars of set_loss)."""
        k = len(log_mass)
        if not (len(mu) == k and len(sigma) == k):
            raise ValueError("log_mass, mu and sigma need the same length")
        arr = [(ctypes.c_double * max(k, 1))(*map(float, v)) for v in (log_mass, mu, sigma)]
        self._sync_stream()
        L.check(L.lib().pmr_set_noise_table(self._ctx, k, *arr))

    def forward(self, modes, want_mass=True):
        """modes: complex64 [B][Np][Np][Np/2+1] -> (mass [B][Nout^3] or None, loss [B][3] f64)."""
        _need(modes, torch.complex64, self.cfg.batch * self.n_modes, "modes")
        mass = (torch.empty(self.cfg.batch, self.n_out3, dtype=torch.float32, device=self.device)
                if want_mass else None)
        loss = torch.empty(self.cfg.batch, 3, dtype=torch.float64, device=self.device)
        self._sync_stream()
        L.check(L.lib().pmr_forward(self._ctx, _ptr(modes), _ptr(mass), _ptr(loss)))
        return mass, loss

    def adjoint(self, loss_bar, mass_bar=None, out=None):
        B = self.cfg.batch
        loss_bar = loss_bar.to(self.device, torch.float64).contiguous()
        _need(loss_bar, torch.float64, B, "loss_bar")
        if mass_bar is not None:
            mass_bar = mass_bar.to(self.device, torch.float32).contiguous()
            _need(mass_bar, torch.float32, B * self.n_out3, "mass_bar")
        if out is None:
            out = torch.empty(B, self.n_modes, dtype=torch.complex64, device=self.device)
        self._sync_stream()
        L.check(L.lib().pmr_adjoint(self._ctx, _ptr(loss_bar), _ptr(mass_bar), _ptr(out)))
        return out

    def profile_begin(self, kernel_class, max_launches=4096):
        """Start event timing of one kernel class (see PMR_PROF_* in pmr.h)."""
        L.check(L.lib().pmr_profile_begin(self._ctx, L.PROF[kernel_class], int(max_launches)))

    def profile_end(self):
        """-> (total_ms, launches, algorithmic_bytes) since profile_begin (synchronises)."""
        ms, n, b = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
        L.check(L.lib().pmr_profile_end(self._ctx, ctypes.byref(ms), ctypes.byref(n),
                                        ctypes.byref(b)))
        return ms.value, n.value, b.value

    def debug(self, what, step=0):
        """Copy an internal buffer of the last forward/adjoint (see PMR_DBG_* in pmr.h)."""
        cfg = self.cfg
        B, np3, nm3, no3 = cfg.batch, cfg.n_part ** 3, cfg.n_mesh ** 3, cfg.n_out ** 3
        spec = {"x": (torch.float64, (B, 3, np3)), "force": (torch.float32, (B, nm3, 3)),
                "sort_ids": (torch.int32, (B * np3,)), "delta_f": (torch.float32, (B, no3)),
                "features": (torch.float32, (2, B, no3)), "mass_r": (torch.float32, (B, no3)),
                "res_s": (torch.float32, (B, no3)), "xbar0": (torch.float32, (B, 3, np3)),
                "pbar0": (torch.float32, (B, 3, np3)), "dbar_f": (torch.float32, (B, no3))}
        dt, shape = spec[what]
        dst = torch.empty(shape, dtype=dt, device=self.device)
        self._sync_stream()
        r = L.lib().pmr_debug_copy(self._ctx, L.DBG[what], int(step), _ptr(dst))
        if r < 0:
            L.check(int(r))
        return dst


class PMForward(torch.autograd.Function):
    """(loss [B], mass [B][Nout^3]) from modes, with the hand-written adjoint (pmr_adjoint)
    as the backward pass.

    Usage: loss, mass = PMForward.apply(modes, pmctx); loss.sum().backward().
    modes: complex64 [B][n_modes] or [B][Np][Np][Np/2+1]; the gradient has the same shape
    (dL/dRe + i dL/dIm, PyTorch's convention for real losses of complex tensors). The context
    keeps the state of one forward only: a backward after another forward on the same context
    raises PmrError with status PMR_E_STATE instead of returning that forward's gradient."""

    @staticmethod
    def forward(ctx, modes, pmctx):
        flat = modes.detach().reshape(pmctx.cfg.batch, -1).contiguous()
        mass, loss = pmctx.forward(flat)
        ctx.pmctx = pmctx
        ctx.generation = pmctx.forward_count()
        ctx.modes_shape = modes.shape
        ctx.set_materialize_grads(False)
        return loss[:, 0].clone(), mass

    @staticmethod
    def backward(ctx, loss_bar, mass_bar):
        pm = ctx.pmctx
        if pm.forward_count() != ctx.generation:
            raise L.PmrError("PMForward.backward: a later forward on the same context replaced "
                             "the state of this one (PMR_E_STATE)", L.PMR_E_STATE)
        if loss_bar is None:
            loss_bar = torch.zeros(pm.cfg.batch, dtype=torch.float64, device=pm.device)
        g = pm.adjoint(loss_bar, mass_bar)
        return g.reshape(ctx.modes_shape), None


# ---------------------------------------------------------------- primitives
def fft_get_tile(n, pass_):
    """(columns, threads, staging) of the strided FFT pass `pass_` (PMR_FFT_YPASS or
    PMR_FFT_XPASS) for size n."""
    c, t, s = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    L.check(L.lib().pmr_fft_get_tile(n, pass_, ctypes.byref(c), ctypes.byref(t), ctypes.byref(s)))
    return c.value, t.value, s.value


def fft_set_tile(n, pass_, columns, threads, staging):
    L.check(L.lib().pmr_fft_set_tile(n, pass_, columns, threads, staging))


def fft_get_slab(n):
    """kz-slab width of the force transforms on an n^3 mesh (0: off)."""
    c = ctypes.c_int()
    L.check(L.lib().pmr_fft_get_slab(n, ctypes.byref(c)))
    return c.value


def fft_set_slab(n, columns):
    L.check(L.lib().pmr_fft_set_slab(n, columns))


def paint_get_rows(n, channels):
    """Rows per wavefront of the CIC paints on an n^3 mesh (0: the default rule)."""
    c = ctypes.c_int()
    L.check(L.lib().pmr_paint_get_rows(n, channels, ctypes.byref(c)))
    return c.value


def paint_set_rows(n, channels, rows):
    L.check(L.lib().pmr_paint_set_rows(n, channels, rows))


def fft_r2c(x):
    """Unnormalised 3-D real FFT of [B][n][n][n] float32 -> complex64 [B][n][n][n/2+1]."""
    B, n = x.shape[0], x.shape[-1]
    x = x.contiguous()
    out = torch.empty(B, n, n, n // 2 + 1, dtype=torch.complex64, device=x.device)
    L.check(L.lib().pmr_fft_r2c(n, B, _ptr(x), _ptr(out), _stream()))
    return out


def fft_c2r(X):
    """Inverse 3-D real FFT (with 1/n^3) of complex64 [B][n][n][n/2+1] -> float32."""
    B, n = X.shape[0], X.shape[1]
    scratch = X.contiguous().clone()
    out = torch.empty(B, n, n, n, dtype=torch.float32, device=X.device)
    L.check(L.lib().pmr_fft_c2r(n, B, _ptr(scratch), _ptr(out), _stream()))
    return out


def cic_sort(x, n_mesh, box):
    """x: float64 [B][3][Np^3] -> (keys_sorted, ids_sorted, row_start) as int32 tensors
    (bit patterns of the u32 outputs)."""
    B, np3 = x.shape[0], x.shape[2]
    n_part = round(np3 ** (1 / 3))
    total = B * np3
    scratch_n = int(L.lib().pmr_sort_scratch_bytes(total, n_mesh, B))
    scratch = torch.empty(scratch_n, dtype=torch.uint8, device=x.device)
    keys = torch.empty(total, dtype=torch.int32, device=x.device)
    ids = torch.empty(total, dtype=torch.int32, device=x.device)
    rows = torch.empty(B * n_mesh * n_mesh + 1, dtype=torch.int32, device=x.device)
    L.check(L.lib().pmr_cic_sort(n_part, n_mesh, B, float(box), _ptr(x.contiguous()), _ptr(keys),
                                 _ptr(ids), _ptr(rows), _ptr(scratch), scratch_n, _stream()))
    return keys, ids, rows


def cic_paint(x, keys, ids, rows, n_mesh, box, mass=1.0, bias=0.0):
    """CIC density of positions x (float64 [B][3][Np^3]) from the outputs of cic_sort."""
    B, np3 = x.shape[0], x.shape[2]
    n_part = round(np3 ** (1 / 3))
    out = torch.empty(B, n_mesh ** 3, dtype=torch.float32, device=x.device)
    scratch = torch.empty(B * np3 * 12, dtype=torch.uint8, device=x.device)
    L.check(L.lib().pmr_cic_paint(n_part, n_mesh, B, float(box), _ptr(x.contiguous()), _ptr(keys),
                                  _ptr(ids), _ptr(rows), float(mass), float(bias), _ptr(out),
                                  _ptr(scratch), scratch.numel(), _stream()))
    return out


class GradientGraph:
    """A gradient evaluation (pmr_forward + pmr_adjoint) captured once as a HIP graph and
    replayed. Inputs and outputs are fixed device buffers: write new modes into
    `self.modes` (and loss_bar into `self.loss_bar`) before `replay()`; read `self.loss`
    and `self.grad` after it. Loss parameters live in device memory, so a new
    pmr_set_loss (anneal stage) is picked up by the next replay without recapture.

    The library enqueues only kernels and device-to-device copies (no memsets), so the
    captured graph replays exactly what the eager calls do.

    With `params` (one LossParams or a list) the loss parameters live in a device buffer
    `self.params` [B][7]: `set_params` writes new stage values into it with a stream-ordered
    copy and applies them with pmr_set_loss_device on the stream, once (the data term of the
    target is recomputed there), so an anneal stage changes between replays without a host
    synchronisation and without recapture. With capture_params=True the graph itself also
    contains pmr_set_loss_device on that buffer, so every replay reads the buffer as it is
    (at the cost of recomputing the data term in every replay).
    """

    def __init__(self, pmctx, modes, warmup=1, params=None, capture_params=False):
        self.pm = pmctx
        B = pmctx.cfg.batch
        self.modes = modes.clone().contiguous()
        self.params = None
        self.capture_params = bool(capture_params)
        if params is not None:
            self.params = torch.tensor(loss_param_rows(params, B), dtype=torch.float64,
                                       device=pmctx.device)
            pmctx.set_loss_device(self.params)
        self.loss_bar = torch.ones(B, dtype=torch.float64, device=pmctx.device)
        self.loss = torch.empty(B, 3, dtype=torch.float64, device=pmctx.device)
        self.grad = torch.empty(B, pmctx.n_modes, dtype=torch.complex64, device=pmctx.device)
        s = torch.cuda.Stream(device=pmctx.device)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self._enqueue()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._enqueue()
        torch.cuda.synchronize()

    def set_params(self, params):
        """New loss parameters for the next replays (captured with `params` only)."""
        if self.params is None:
            raise ValueError("GradientGraph was captured without device loss parameters")
        rows = torch.tensor(loss_param_rows(params, self.pm.cfg.batch), dtype=torch.float64)
        self.params.copy_(rows.pin_memory(), non_blocking=True)
        if not self.capture_params:
            self.pm.set_loss_device(self.params)

    def _enqueue(self):
        pm = self.pm
        pm._sync_stream()
        if self.params is not None and self.capture_params:
            L.check(L.lib().pmr_set_loss_device(pm._ctx, _ptr(self.params)))
        L.check(L.lib().pmr_forward(pm._ctx, _ptr(self.modes), None, _ptr(self.loss)))
        L.check(L.lib().pmr_adjoint(pm._ctx, _ptr(self.loss_bar), None, _ptr(self.grad)))

    def replay(self):
        self.graph.replay()
        # later eager calls must see the library's stream, not the capture stream
        self.pm._sync_stream()
        return self.loss, self.grad
