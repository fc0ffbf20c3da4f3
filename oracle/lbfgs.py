"""Oracle: the reconstruction driver -- limited-memory BFGS over the linear modes with a
backtracking line search, run over the smoothing / M0 anneal schedule (Sec. 5.2) -- in
FP64 with plain numpy.

TEST INFRASTRUCTURE ONLY. Nothing in the product imports this package.

What is computed
----------------
The parameters are all stored real and imaginary parts of the modes (the gradient
convention of model.py), so the inner product of two mode arrays a, b is
Re sum conj(a) b over the stored entries.

L-BFGS (Sec. 5.2 names the method; Nocedal and Wright, Numerical Optimization, Alg. 7.4
and 7.5, is the standard statement): the direction is d = -H g, with H the inverse-Hessian
approximation built from the m newest pairs s = x_{k+1} - x_k, y = g_{k+1} - g_k by the
two-loop recursion, starting from H0 = gamma I with gamma = s.y / y.y of the newest pair.

Readings (the paper gives no parameters of its optimiser):
* history m = 10;
* the first iteration of a stage (empty history) steps along -g with step length 1/|g|
  (a unit move in parameter space);
* backtracking line search from step 1 (1/|g| without history), halving until the Armijo
  condition f(x + t d) <= f(x) + c1 t g.d with c1 = 1e-4 holds, at most 30 halvings
  (failure ends the stage);
* a pair enters the history only if s.y > 1e-10 |s| |y| (curvature);
* if d is not a descent direction the history is cleared and -g is used;
* a stage ends when the loss decreases by less than rel_tol = 1e-3 of its value between
  successive iterations (the paper's 0.1% rule, Sec. 5.3), at a zero gradient, or after
  max_iter iterations; the rule is not applied to a unit-length step taken without
  history (its decrease says nothing about convergence);
* the anneal stages run in order, each starting from the previous stage's optimum with an
  empty history.
"""
import numpy as np

HISTORY = 10
C1 = 1e-4
MAX_HALVINGS = 30
CURVATURE_EPS = 1e-10
REL_TOL = 1e-3


def inner(a, b):
    """Inner product of two parameter arrays (complex modes: real and imaginary parts)."""
    return float(np.sum(a.real * b.real) + np.sum(a.imag * b.imag)) if np.iscomplexobj(a) \
        else float(np.sum(a * b))


def two_loop(g, S, Y):
    """H g for the L-BFGS inverse-Hessian approximation of the pairs (S[i], Y[i]),
    oldest first (Nocedal and Wright, Alg. 7.4)."""
    q = g.copy()
    alpha = []
    for s, y in zip(reversed(S), reversed(Y)):
        a = inner(s, q) / inner(y, s)
        q = q - a * y
        alpha.append(a)
    gamma = inner(S[-1], Y[-1]) / inner(Y[-1], Y[-1]) if S else 1.0
    r = gamma * q
    for (s, y), a in zip(zip(S, Y), reversed(alpha)):
        b = inner(y, r) / inner(y, s)
        r = r + (a - b) * s
    return r


def dense_inverse_hessian(S, Y, n):
    """The same approximation as an explicit n x n matrix (BFGS update of H0 = gamma I)."""
    gamma = inner(S[-1], Y[-1]) / inner(Y[-1], Y[-1]) if S else 1.0
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / inner(y, s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


def minimize(fg, x0, max_iter=100, m=HISTORY, rel_tol=REL_TOL, log=None):
    """L-BFGS from x0 (one anneal stage). fg(x) -> (f, g). Returns (x, f, info) with info
    holding the per-iteration losses, the number of evaluations and the stop reason."""
    x = x0.copy()
    f, g = fg(x)
    S, Y = [], []
    losses, evals, reason = [f], 1, "max_iter"
    for it in range(max_iter):
        if inner(g, g) == 0.0:
            reason = "stationary"
            break
        d = -two_loop(g, S, Y)
        gd = inner(g, d)
        if gd >= 0.0:
            S, Y = [], []
            d = -g
            gd = inner(g, d)
        probe = not S  # unit-length step without history
        t = 1.0 if S else 1.0 / np.sqrt(inner(g, g))
        ok = False
        for _ in range(MAX_HALVINGS + 1):
            xn = x + t * d
            fn, gn = fg(xn)
            evals += 1
            if fn <= f + C1 * t * gd:
                ok = True
                break
            t *= 0.5
        if not ok:
            reason = "line_search"
            break
        s, y = xn - x, gn - g
        sy = inner(s, y)
        if sy > CURVATURE_EPS * np.sqrt(inner(s, s) * inner(y, y)):
            S.append(s)
            Y.append(y)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        rel = (f - fn) / abs(f) if f != 0.0 else 0.0
        x, f, g = xn, fn, gn
        losses.append(f)
        if log:
            log(it, f, t, evals)
        if rel < rel_tol and not probe:
            reason = "converged"
            break
    return x, f, {"losses": losses, "evals": evals, "reason": reason}


def reconstruct(stages, make_fg, x0, max_iter=100, log=None):
    """Runs minimize over the anneal stages in order. stages: list of parameter sets;
    make_fg(stage) -> fg. Returns (x, per-stage info)."""
    x = x0
    infos = []
    for st in stages:
        x, f, info = minimize(make_fg(st), x, max_iter=max_iter, log=log)
        info["stage"] = st
        info["loss"] = f
        infos.append(info)
    return x, infos
