"""Oracle: the differentiable forward model (linear modes -> halo-mass field -> loss)
and its hand-transposed gradient, all in FP64 with plain numpy.

TEST INFRASTRUCTURE ONLY. Nothing in the product imports this package.

What is computed, in the paper's order
--------------------------------------
1. Prior on the linear modes (Sec. 5.1, Eq. priorpdf): 0.5 * sum over the full
   spectrum of |s|^2 / S(k), S = <|s|^2> (diagonal in k).
2. Dynamics (Sec. 3, Sec. 5): Zel'dovich displacement at a0, then an n-step
   particle-mesh kick-drift-kick evolution with FastPM-style linear-exact factors.
   (The paper starts from 2LPT: ic_order = 2 adds the second-order displacement.)
3. Halo model (Sec. 2.1, Sec. 2.2): features (delta_0, delta_R1, delta_R1 - delta_R2) of
   the final CIC density, then either a per-voxel fully connected network with
   mass = softplus(output) (halo_model = HALO_SINGLE), or the paper's two networks
   (HALO_TWO): a position network on the features of the 3 x 3 x 3 neighbourhood whose
   logistic output (sharpness a, Eq. logistic) is multiplied by a mass network on the
   voxel's own features (Sec. 2, Sec. 2.1).
4. Likelihood (Sec. 5.1, Eqs. var, probnoise, loss): x = log(M_R + M0) with M_R the
   Gaussian-smoothed mass; residual (mu + x - x_data) / (2 sigma_N); f_eff = 1.
   Residual smoothing anneal (Sec. 5.2): the residual is Gaussian-smoothed on R_sm
   before squaring; R_sm = 0 is the identity.
5. Gradient of the loss with respect to the stored linear modes (Sec. 5.2: the
   optimiser needs dL/ds for all modes), by transposing every step by hand.

Gradient convention: modes are stored in rfft layout and every stored real and
imaginary part is a parameter; G = dL/dRe(s) + i dL/dIm(s), so that
dL = sum_stored Re(G) Re(ds) + Im(G) Im(ds).

Checks against the paper or mathematics live in tests/test_oracle_*.py.
"""
import numpy as np

from . import cosmology as cos
from . import mesh as M

LOSS_DENSITY_L2 = 0
LOSS_LOGNORMAL = 1
HALO_SINGLE = 0
HALO_TWO = 1


class Config:
    def __init__(self, box, n_part, n_mesh, n_out, n_steps, a0=0.1, a1=1.0,
                 omega_m=cos.OMEGA_M_PAPER, R1=1.0, R2=2.0, loss_kind=LOSS_LOGNORMAL,
                 ic_order=1, halo_model=HALO_SINGLE):
        self.box = float(box)
        self.n_part, self.n_mesh, self.n_out = int(n_part), int(n_mesh), int(n_out)
        self.n_steps = int(n_steps)
        self.a0, self.a1, self.omega_m = float(a0), float(a1), float(omega_m)
        self.R1, self.R2 = float(R1), float(R2)
        self.loss_kind = loss_kind
        self.ic_order = int(ic_order)  # 1: Zel'dovich, 2: second-order LPT
        self.halo_model = int(halo_model)
        self.fac = cos.kdk_factors(self.a0, self.a1, self.n_steps, self.omega_m)


def default_params(**kw):
    p = dict(M0=1.0, mu=0.0, sigma_N=0.5, R_mass=3.0, R_sm=0.0, prior_weight=1.0,
             logistic_a=3.0)
    p.update(kw)
    return p


# ------------------------------------------------------------------ prior

def prior_loss(s, inv_S):
    """0.5 * sum_full |P s|^2 / S (Eq. priorpdf exponent), summed over stored modes with
    their full-spectrum multiplicity."""
    n = s.shape[0]
    ps = M.hermitian_project(s)
    return 0.5 * np.sum(M.hermitian_weight(n) * np.abs(ps) ** 2 * inv_S)


def prior_grad(s, inv_S):
    n = s.shape[0]
    ps = M.hermitian_project(s)
    return M.hermitian_weight(n) * ps * inv_S


# ------------------------------------------------------------------ dynamics

HESS_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
LPT2_D = 3.0 / 7.0  # |D2| / D1^2 (second-order growth, the Omega_m = 1 relation)


def lpt2_source(phi):
    """Second-order source sum_{a<b} (phi_aa phi_bb - phi_ab^2) from the six phi_{,ab}
    (in HESS_PAIRS order)."""
    xx, yy, zz, xy, xz, yz = phi
    return xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz


def zeldovich(cfg, s, full=False):
    """Initial conditions on the particle lattice q.
    First order (Zel'dovich): Psi_a = irfft(i k_a / k^2 * P s); x0 = wrap(q + D Psi),
    p0 = G_p Psi, with D, G_p at a0.
    Second order (ic_order = 2; the paper's initial conditions are 2LPT, Sec. 3; the
    standard second-order Lagrangian solution is the reading): with phi_{,ab} =
    irfft(k_a k_b / k^2 * P s) the second derivatives of the potential of the linear field
    and S = sum_{a<b} (phi_aa phi_bb - phi_ab^2), Psi2_a = irfft(i k_a / k^2 * rfft(S));
    the second-order displacement is -D2 * Psi2 with D2 = -(3/7) D^2, so
    x0 = wrap(q + D Psi + (3/7) D^2 Psi2), p0 = G_p Psi + (6/7) D G_p Psi2 (the momentum
    factor of D^2 is 2 D G_p, since G_p = a^3 E dD/da).
    full: also return the intermediates the adjoint needs."""
    n = cfg.n_part
    ps = M.hermitian_project(s)
    psi = np.stack([M.irfft3(M.gradient_multiplier(n, cfg.box, a) * ps, n).ravel()
                    for a in range(3)])
    q = M.lattice_positions(n, cfg.box, cfg.n_mesh)
    D, Gp = cfg.fac["D0"], cfg.fac["Gp0"]
    extra = {}
    if cfg.ic_order == 2:
        phi = [M.irfft3(M.hessian_multiplier(n, cfg.box, a, b) * ps, n) for a, b in HESS_PAIRS]
        S = lpt2_source(phi)
        Sh = M.rfft3(S)
        psi2 = np.stack([M.irfft3(M.gradient_multiplier(n, cfg.box, a) * Sh, n).ravel()
                         for a in range(3)])
        x0 = M.wrap(q + D * psi + LPT2_D * D * D * psi2, cfg.box)
        p0 = Gp * psi + 2.0 * LPT2_D * D * Gp * psi2
        extra = {"phi": phi, "S": S, "psi2": psi2}
    else:
        x0 = M.wrap(q + D * psi, cfg.box)
        p0 = Gp * psi
    if full:
        return x0, p0, psi, extra
    return x0, p0, psi


def density(cfg, x, n):
    """CIC density contrast on an n^3 mesh; each particle has mass (n / n_part)^3 so that
    the mean density is 1."""
    m = (n / cfg.n_part) ** 3
    return M.cic_paint(x, n, cfg.box, np.full(x.shape[1], m)) - 1.0


def force_meshes(cfg, delta):
    """Force meshes F_a = irfft(i k_a / k^2 * rfft(delta)), a = x, y, z."""
    n = delta.shape[0]
    dk = M.rfft3(delta)
    return np.stack([M.irfft3(M.gradient_multiplier(n, cfg.box, a) * dk, n) for a in range(3)])


def pm_forward(cfg, x0, p0):
    """n kick-drift-kick steps. Force i is evaluated at x_i; the kick around x_i merges the
    two half kicks; the force at the final time would only feed the final half kick of
    the momentum, which nothing downstream uses, so it is not evaluated.
    Returns the list of positions x_0..x_n, momenta p_{1/2}.., force meshes and
    interpolated forces."""
    n_m = cfg.n_mesh
    xs, ps, Fm, Fp = [x0], [], [], []
    x, p = x0, p0
    for i in range(cfg.n_steps):
        delta = density(cfg, x, n_m)
        F = force_meshes(cfg, delta)
        Fx = M.cic_readout(x, n_m, cfg.box, F)
        p = p + cfg.fac["kick"][i] * Fx
        x = M.wrap(x + cfg.fac["drift"][i] * p, cfg.box)
        Fm.append(F)
        Fp.append(Fx)
        ps.append(p)
        xs.append(x)
    return xs, ps, Fm, Fp


# ------------------------------------------------------------------ halo model

def relu(v):
    return np.maximum(v, 0.0)  # Eq. relu


def softplus(y):
    return np.maximum(y, 0.0) + np.log1p(np.exp(-np.abs(y)))


def sigmoid(y):
    return 0.5 * (1.0 + np.tanh(0.5 * y))


def features(cfg, delta_f):
    """Sec. 2.2: (delta_0, delta_R1, delta_R1 - delta_R2) with Gaussian smoothing."""
    n = delta_f.shape[0]
    dk = M.rfft3(delta_f)
    d1 = M.irfft3(M.gaussian_multiplier(n, cfg.box, cfg.R1) * dk, n)
    d2 = M.irfft3(M.gaussian_multiplier(n, cfg.box, cfg.R2) * dk, n)
    return np.stack([delta_f, d1, d1 - d2])


def mlp_forward(w, f):
    """Per-voxel network (Sec. 2.1): two ReLU hidden layers, linear output, then softplus.
    f: (3, V) -> dict of pre-activations and the mass M (V,)."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(w[k], dtype=np.float64)
                              for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    a1 = W1 @ f + b1[:, None]
    h1 = relu(a1)
    a2 = W2 @ h1 + b2[:, None]
    h2 = relu(a2)
    y = (W3 @ h2 + b3[:, None])[0]
    return {"a1": a1, "a2": a2, "y": y, "mass": softplus(y)}


def mlp_backward(w, cache, mass_bar):
    """Input gradient of the network (weights frozen): returns f_bar (3, V)."""
    W1, W2, W3 = (np.asarray(w[k], dtype=np.float64) for k in ("W1", "W2", "W3"))
    y_bar = mass_bar * sigmoid(cache["y"])
    a2_bar = (W3[0][:, None] * y_bar[None, :]) * (cache["a2"] > 0)
    a1_bar = (W2.T @ a2_bar) * (cache["a1"] > 0)
    return W1.T @ a1_bar


# The paper's two-network model (Sec. 2: model = NNp x NNm; Sec. 2.1: architecture).

# Offsets of the 3 x 3 x 3 neighbourhood; position-network feature c * 27 + o holds
# feature field c at the voxel displaced by STENCIL[o] (periodic mesh).
STENCIL = tuple((dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1))


def elu(v):
    """Eq. elu: v for v > 0, exp(v) - 1 otherwise."""
    return np.where(v > 0, v, np.expm1(np.minimum(v, 0.0)))


def logistic(x, a):
    """Eq. logistic: 1 / (1 + exp(-a x)) (written with tanh, which cannot overflow)."""
    return 0.5 * (1.0 + np.tanh(0.5 * a * x))


def stencil_features(f):
    """(3, n, n, n) feature fields -> (81, n^3): the values of each field on the voxel's
    3 x 3 x 3 neighbourhood (Sec. 2.2: the position network sees 3 x 27 = 81 features)."""
    rows = []
    for c in range(3):
        for d in STENCIL:
            rows.append(np.roll(f[c], shift=(-d[0], -d[1], -d[2]), axis=(0, 1, 2)).ravel())
    return np.stack(rows)


def stencil_adjoint(Fbar, n):
    """Transpose of stencil_features: (81, n^3) -> (3, n, n, n)."""
    out = np.zeros((3, n, n, n))
    for c in range(3):
        for o, d in enumerate(STENCIL):
            out[c] += np.roll(Fbar[c * 27 + o].reshape(n, n, n), shift=d, axis=(0, 1, 2))
    return out


def _w(net, k):
    return np.asarray(net[k], dtype=np.float64)


def two_net_forward(nets, f, a):
    """NNp: 81 features -> 50 -> 30 (ReLU) -> 1, then logistic(., a) (the position mask);
    NNm: 3 features -> 20 -> 10 (ELU) -> 1, linear (the mass); mass = NNp x NNm.
    f: (3, n, n, n). Returns a dict of pre-activations and the mass (n^3,)."""
    p, m = nets["nnp"], nets["nnm"]
    F = stencil_features(f)
    a1 = _w(p, "W1") @ F + _w(p, "b1")[:, None]
    a2 = _w(p, "W2") @ relu(a1) + _w(p, "b2")[:, None]
    y = (_w(p, "W3") @ relu(a2) + _w(p, "b3")[:, None])[0]
    pos = logistic(y, a)
    f3 = f.reshape(3, -1)
    z1 = _w(m, "W1") @ f3 + _w(m, "b1")[:, None]
    z2 = _w(m, "W2") @ elu(z1) + _w(m, "b2")[:, None]
    mm = (_w(m, "W3") @ elu(z2) + _w(m, "b3")[:, None])[0]
    return {"a1": a1, "a2": a2, "y": y, "pos": pos, "z1": z1, "z2": z2, "m": mm,
            "mass": pos * mm}


def two_net_backward(nets, cache, mass_bar, a, n):
    """Input gradient of the two-network model (weights frozen): (3, n, n, n)."""
    p, m = nets["nnp"], nets["nnm"]
    pos_bar = mass_bar * cache["m"]
    m_bar = mass_bar * cache["pos"]
    pos = cache["pos"]
    y_bar = pos_bar * a * pos * (1.0 - pos)  # d logistic(y, a) / dy
    a2_bar = (_w(p, "W3")[0][:, None] * y_bar[None, :]) * (cache["a2"] > 0)
    a1_bar = (_w(p, "W2").T @ a2_bar) * (cache["a1"] > 0)
    fbar = stencil_adjoint(_w(p, "W1").T @ a1_bar, n)
    delu = lambda z: np.where(z > 0, 1.0, np.exp(np.minimum(z, 0.0)))  # noqa: E731
    z2_bar = (_w(m, "W3")[0][:, None] * m_bar[None, :]) * delu(cache["z2"])
    z1_bar = (_w(m, "W2").T @ z2_bar) * delu(cache["z1"])
    return fbar + (_w(m, "W1").T @ z1_bar).reshape(3, n, n, n)


def smooth(cfg, field, R):
    n = field.shape[0]
    return M.apply_multiplier(field, M.gaussian_multiplier(n, cfg.box, R))


def target_x(cfg, mass_target, params):
    """x_data = log(G_{R_mass} * M_target + M0) (Eq. var)."""
    return np.log(smooth(cfg, mass_target, params["R_mass"]) + params["M0"])


def noise_fields(cfg, mass_target, params):
    """Per-cell offset and width (mu_N, sigma_N) of the displaced log-normal noise (Eq.
    probnoise). Sec. 5.1: both depend on the smoothed data mass at the cell. Without a table
    they are the scalars of params; with params["noise_table"] = (t, mu, sigma) -- nodes t
    ascending in log(M_R,data), natural log -- they are the linear interpolation of the
    table at log(M_R,data), held constant beyond the end nodes (reading: the paper fits one
    (mu, sigma) per mass bin; interpolating between bins keeps the loss continuous in the
    data)."""
    tab = params.get("noise_table")
    if tab is None:
        return params["mu"], params["sigma_N"]
    t_nodes, mu_nodes, sig_nodes = (np.asarray(v, np.float64) for v in tab)
    MRd = smooth(cfg, mass_target, params["R_mass"])
    with np.errstate(divide="ignore"):
        t = np.log(np.maximum(MRd, 0.0))
    return np.interp(t, t_nodes, mu_nodes), np.interp(t, t_nodes, sig_nodes)


# ------------------------------------------------------------------ forward

def forward(cfg, s, inv_S, target, params, mlp=None):
    """Full forward model and loss for one realisation. Returns a dict of intermediates."""
    out = {}
    x0, p0, psi, lpt2 = zeldovich(cfg, s, full=True)
    xs, ps, Fm, Fp = pm_forward(cfg, x0, p0)
    out.update(x0=x0, p0=p0, psi=psi, lpt2=lpt2, xs=xs, ps=ps, Fm=Fm, Fp=Fp)
    n_o = cfg.n_out
    delta_f = density(cfg, xs[-1], n_o)
    out["delta_f"] = delta_f
    lp = prior_loss(s, inv_S)
    out["loss_prior"] = lp
    if cfg.loss_kind == LOSS_DENSITY_L2:
        res = delta_f - target
        out["loss_data"] = np.sum(res ** 2)
        out["mass"] = None
    else:
        f = features(cfg, delta_f)
        if cfg.halo_model == HALO_TWO:
            c = two_net_forward(mlp, f, params["logistic_a"])
        else:
            c = mlp_forward(mlp, f.reshape(3, -1))
        mass = c["mass"].reshape(n_o, n_o, n_o)
        MR = smooth(cfg, mass, params["R_mass"])
        xd = target_x(cfg, target, params)
        xm = np.log(MR + params["M0"])
        mu_n, sig_n = noise_fields(cfg, target, params)
        r = (mu_n + xm - xd) / (2.0 * sig_n)
        rs = smooth(cfg, r, params["R_sm"])
        out.update(features=f, mlp_cache=c, mass=mass, MR=MR, r=r, rs=rs)
        out["loss_data"] = np.sum(rs ** 2)
    out["loss"] = params["prior_weight"] * lp + out["loss_data"]
    return out


# ------------------------------------------------------------------ adjoint

def force_adjoint_mesh(cfg, Fbar):
    """Transpose of delta -> F_a: delta_bar = irfft(sum_a conj(i k_a / k^2) rfft(Fbar_a))."""
    n = Fbar.shape[1]
    acc = 0.0
    for a in range(3):
        acc = acc + np.conj(M.gradient_multiplier(n, cfg.box, a)) * M.rfft3(Fbar[a])
    return M.irfft3(acc, n)


def density_adjoint_positions(cfg, x, n, delta_bar):
    """Transpose of x -> CIC density on an n^3 mesh, with respect to positions."""
    m = (n / cfg.n_part) ** 3
    return m * M.cic_readout_grad(x, n, cfg.box, delta_bar)[0]


def pm_adjoint(cfg, fwd, x_bar_final):
    """Reverse the kick-drift-kick steps. Returns (x0_bar, p0_bar)."""
    n_m = cfg.n_mesh
    xs, Fm = fwd["xs"], fwd["Fm"]
    x_bar = x_bar_final.copy()
    p_bar = np.zeros_like(x_bar)
    for i in reversed(range(cfg.n_steps)):
        # drift: x_{i+1} = x_i + drift_i * p_{i+1/2}  (the periodic wrap has unit derivative)
        p_bar = p_bar + cfg.fac["drift"][i] * x_bar
        # kick: p_{i+1/2} = p_{i-1/2} + kick_i * F(x_i)
        F_bar = cfg.fac["kick"][i] * p_bar
        x = xs[i]
        # (i) readout-position term with the stored force meshes
        g = M.cic_readout_grad(x, n_m, cfg.box, Fm[i])  # (3 comps, 3 axes, P)
        x_bar = x_bar + np.einsum("cp,cap->ap", F_bar, g)
        # (ii) readout-mesh term: paint F_bar, transpose the force operator
        Fbar_mesh = M.cic_paint(x, n_m, cfg.box, F_bar)
        delta_bar = force_adjoint_mesh(cfg, Fbar_mesh)
        # (iii) paint-position term
        x_bar = x_bar + density_adjoint_positions(cfg, x, n_m, delta_bar)
    return x_bar, p_bar


def zeldovich_adjoint(cfg, x0_bar, p0_bar, lpt2=None):
    """Gradient with respect to the stored modes from (x0_bar, p0_bar) (without prior);
    lpt2: the second-order intermediates of zeldovich(..., full=True) when ic_order = 2.
    A real-space map f -> irfft(m rfft(f)) has the transpose g -> irfft(conj(m) rfft(g));
    a map from the modes, P s -> irfft(m P s), contributes w conj(m) rfft(g) / n^3."""
    n = cfg.n_part
    D, Gp = cfg.fac["D0"], cfg.fac["Gp0"]
    psi_bar = D * x0_bar + Gp * p0_bar
    g = 0.0
    for a in range(3):
        g = g + np.conj(M.gradient_multiplier(n, cfg.box, a)) * M.rfft3(
            psi_bar[a].reshape(n, n, n))
    if cfg.ic_order == 2:
        psi2_bar = LPT2_D * D * D * x0_bar + 2.0 * LPT2_D * D * Gp * p0_bar
        sb = 0.0
        for a in range(3):
            sb = sb + np.conj(M.gradient_multiplier(n, cfg.box, a)) * M.rfft3(
                psi2_bar[a].reshape(n, n, n))
        S_bar = M.irfft3(sb, n)
        xx, yy, zz, xy, xz, yz = lpt2["phi"]
        phi_bar = [(yy + zz) * S_bar, (xx + zz) * S_bar, (xx + yy) * S_bar,
                   -2.0 * xy * S_bar, -2.0 * xz * S_bar, -2.0 * yz * S_bar]
        for (a, b), pb in zip(HESS_PAIRS, phi_bar):
            g = g + M.hessian_multiplier(n, cfg.box, a, b) * M.rfft3(pb)
    G = np.array(M.hermitian_weight(n) * g / n ** 3)
    G[0, 0, 0] = 0.0
    return G


def halo_adjoint(cfg, fwd, target, params, mlp, loss_bar=1.0):
    """Loss -> final density contrast adjoint (log-normal likelihood, network, features)."""
    rs_bar = 2.0 * fwd["rs"] * loss_bar
    r_bar = smooth(cfg, rs_bar, params["R_sm"])
    x_bar = r_bar / (2.0 * noise_fields(cfg, target, params)[1])
    MR_bar = x_bar / (fwd["MR"] + params["M0"])
    mass_bar = smooth(cfg, MR_bar, params["R_mass"])
    n_o = cfg.n_out
    if cfg.halo_model == HALO_TWO:
        fbar = two_net_backward(mlp, fwd["mlp_cache"], mass_bar.ravel(), params["logistic_a"],
                                n_o)
    else:
        fbar = mlp_backward(mlp, fwd["mlp_cache"], mass_bar.ravel()).reshape(3, n_o, n_o, n_o)
    g1 = M.gaussian_multiplier(n_o, cfg.box, cfg.R1)
    g2 = M.gaussian_multiplier(n_o, cfg.box, cfg.R2)
    spec = g1 * M.rfft3(fbar[1] + fbar[2]) - g2 * M.rfft3(fbar[2])
    return fbar[0] + M.irfft3(spec, n_o)


def gradient(cfg, s, inv_S, target, params, mlp=None, loss_bar=1.0):
    """Loss and its gradient with respect to the stored modes. Returns (fwd dict, G)."""
    fwd = forward(cfg, s, inv_S, target, params, mlp)
    if cfg.loss_kind == LOSS_DENSITY_L2:
        delta_bar = 2.0 * (fwd["delta_f"] - target) * loss_bar
    else:
        delta_bar = halo_adjoint(cfg, fwd, target, params, mlp, loss_bar)
    fwd["delta_f_bar"] = delta_bar
    xbar_n = density_adjoint_positions(cfg, fwd["xs"][-1], cfg.n_out, delta_bar)
    x0_bar, p0_bar = pm_adjoint(cfg, fwd, xbar_n)
    fwd["x0_bar"], fwd["p0_bar"] = x0_bar, p0_bar
    G = zeldovich_adjoint(cfg, x0_bar, p0_bar, fwd["lpt2"])
    G = G + params["prior_weight"] * loss_bar * prior_grad(s, inv_S)
    return fwd, G


# ------------------------------------------------------------------ inputs

def prior_inv_variance(n, box, power):
    """1 / S(k) with S = <|s(k)|^2> = n^6 P(k) / L^3 for the unnormalised DFT; 0 at k = 0."""
    kv = M.wavevectors(n, box)
    k = np.sqrt(kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2)
    with np.errstate(divide="ignore"):
        S = n ** 6 * power(np.where(k == 0, 1.0, k)) / box ** 3
        inv = 1.0 / S
    inv = np.where(k == 0, 0.0, inv)
    return np.ascontiguousarray(np.broadcast_to(inv, (n, n, n // 2 + 1)))


def linear_modes(white, box, power):
    """Gaussian linear modes with <|s|^2> = S(k): s = rfft(w) * sqrt(P(k) / L^3 * n^3)."""
    n = white.shape[0]
    kv = M.wavevectors(n, box)
    k = np.sqrt(kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2)
    amp = np.sqrt(power(np.where(k == 0, 1.0, k)) * n ** 3 / box ** 3)
    s = M.rfft3(white) * amp
    s[0, 0, 0] = 0.0
    return s
