"""Discrete adjoint of the split exponential Euler scheme (gradient oracle).

Not in the paper: the paper integrates forward only.  This is the exact
reverse-mode derivative of the *discrete* map of eq. (BVAM_SExpE),

    W^{n+1}_s = W^n_s + tau S_s(d_s) F_s,   F_s = d_s (M W^n_s + r w_D,s) + G_s(W^n; p),
    S_s(d) = phi_1(tau d M_1) ... phi_1(tau d M_d),

for the loss L = 1/2 sum_x (u^N - u_target)^2 over grid points (species 0).
With mu_s = tau S_s^T lambda^{n+1}_s the backward recursion is

    lambda^n_s = lambda^{n+1}_s + d_s M^T mu_s + sum_r (dG_r/dW_s) mu_r,
    dL/dd_s   += <lambda^{n+1}_s, tau (dS_s/dd) F_s> + <mu_s, M W^n_s + r w_D,s>,
    dL/dp     += sum_r <mu_r, dG_r/dp>.

dS/dd uses d/dd phi_1(tau d X) = tau X (phi_1 - phi_2)(tau d X), applied
through the same mode products as S (a tangent carried along the chain).
Pinned by the dot-product identity and by central finite differences of L.
"""
from __future__ import annotations

import numpy as np

from . import assemble, reactions
from .phi import eig_tridiag, phi1_scalar, phi2_scalar
from .splitee import SplitEE, mode_product


def _dphi1(c, x):
    """d/dd phi_1(d c) at d with x = d c:  c (phi_1(x) - phi_2(x))."""
    return c * (phi1_scalar(x) - phi2_scalar(x))


def _dense_pair(A, c):
    """phi_1(c A) and its derivative w.r.t. the scalar multiplying c."""
    lam, V, Vinv = eig_tridiag(A)
    x = c * lam
    P = (V * phi1_scalar(x)[None, :]) @ Vinv
    dP = (V * (lam * (phi1_scalar(x) - phi2_scalar(x)))[None, :]) @ Vinv
    return P, dP


def chain(se: SplitEE, s: int):
    """The split action for species s as a list of linear ops in application order.

    Each op is ("mode", L, dL, mu) meaning X x_mu L (dL = d L / d d_s or None)
    or ("had", Phi, dPhi) meaning Phi o X.  Order follows eqs. (ee_*).
    """
    g, A, tau, d = se.geometry, se.A, se.tau, se.diff[s]
    ops = []
    if g in ("disk", "disk_lambda"):
        lam_t, Q, _ = eig_tridiag(A[1])
        c = tau * np.outer(se.grid[0] ** (-2.0 - (se.extent[1] if g == "disk_lambda" else 0.0)), lam_t)
        P, dP = _dense_pair(A[0], tau * d)
        ops = [("mode", Q.T, None, 2), ("had", phi1_scalar(d * c), _dphi1(c, d * c)),
               ("mode", Q, None, 2), ("mode", P, tau * dP, 1)]
    elif g == "sphere":
        lam_t, Q, _ = eig_tridiag(A[0])
        s2 = se.extent[0] ** -2.0
        c = tau * s2 * np.outer(lam_t, np.sin(se.grid[1]) ** -2.0)
        P, dP = _dense_pair(A[1], tau * d * s2)
        ops = [("mode", P, tau * s2 * dP, 2), ("mode", Q.T, None, 1),
               ("had", phi1_scalar(d * c), _dphi1(c, d * c)), ("mode", Q, None, 1)]
    elif g == "ball":
        lam_t, Q, _ = eig_tridiag(A[1])
        lam_p, Vp, Vpinv = eig_tridiag(A[2])
        rinv2 = se.grid[0] ** -2.0
        sinv2 = np.sin(se.grid[2]) ** -2.0
        c3 = tau * np.outer(rinv2, lam_p)[:, None, :] * np.ones((1, se.n[1], 1))
        c2 = tau * rinv2[:, None, None] * lam_t[None, :, None] * sinv2[None, None, :]
        P, dP = _dense_pair(A[0], tau * d)
        ops = [("mode", Vpinv, None, 3), ("had", phi1_scalar(d * c3), _dphi1(c3, d * c3)),
               ("mode", Vp, None, 3), ("mode", Q.T, None, 2),
               ("had", phi1_scalar(d * c2), _dphi1(c2, d * c2)),
               ("mode", Q, None, 2), ("mode", P, tau * dP, 1)]
    elif g == "cylinder":
        lam_t, Q, _ = eig_tridiag(A[1])
        c = tau * np.outer(se.grid[0] ** -2.0, lam_t)[:, :, None] * np.ones((1, 1, se.n[2]))
        P, dP = _dense_pair(A[0], tau * d)
        Pz, dPz = _dense_pair(A[2], tau * d)
        ops = [("mode", Pz, tau * dPz, 3), ("mode", Q.T, None, 2),
               ("had", phi1_scalar(d * c), _dphi1(c, d * c)),
               ("mode", Q, None, 2), ("mode", P, tau * dP, 1)]
    else:
        raise ValueError(g)
    return ops


def apply_chain(ops, X):
    for op in ops:
        X = mode_product(X, op[1], op[3]) if op[0] == "mode" else op[1] * X
    return X


def apply_chain_T(ops, X, rnd=None):
    """S^T X: the transposed ops in reverse order.  ``rnd`` (optional) is
    applied to every intermediate result (used to model a lower-precision
    evaluation of the same recursion)."""
    for op in reversed(ops):
        X = mode_product(X, op[1].T, op[3]) if op[0] == "mode" else op[1] * X
        if rnd is not None:
            X = rnd(X)
    return X


def apply_chain_dd(ops, X):
    """(dS/dd) X by forward tangent propagation through the chain."""
    x, t = X, np.zeros_like(X)
    for op in ops:
        if op[0] == "mode":
            t = mode_product(t, op[1], op[3])
            if op[2] is not None:
                t = t + mode_product(x, op[2], op[3])
            x = mode_product(x, op[1], op[3])
        else:
            t = op[1] * t + op[2] * x
            x = op[1] * x
    return t


def param_derivative(kind, U, params):
    """dG_r/dp_q pointwise, list over r of list over q.

    Schnakenberg p = (a, b); AIS3 p = (a, b, kappa, mu) with
    G = (a - u + u^2 v - kappa u w, b - u^2 v, mu (u - w)); scaled
    Schnakenberg p = (a, b, gamma) with G = gamma (a - u + u^2 v, b - u^2 v).
    """
    one = np.ones_like(U[0])
    zero = np.zeros_like(U[0])
    if kind == "schnakenberg":
        return [[one, zero], [zero, one]]
    if kind == "ais3":
        u, _, w = U
        return [[one, zero, -u * w, zero], [zero, one, zero, zero], [zero, zero, zero, u - w]]
    if kind == "schnakenberg_scaled":
        u, v = U
        a, b, gam = params
        return [[gam * one, zero, a - u + u * u * v], [zero, gam * one, b - u * u * v]]
    raise NotImplementedError(kind)


def loss_and_grad(workload, W0s, target, steps, n=None, diff=None, params=None, w_dirichlet=None,
                  round_to=None):
    """L and dL/d(W0, d_s, params) for species-list W0s (arrays [i,j,..]).

    ``w_dirichlet`` (per species) is the boundary value at z_* of the
    cylinder; the lifted term d_s r w_D then enters F and dL/dd_s.
    ``round_to`` (a NumPy float type, default None = exact FP64) rounds the
    reverse sweep's stored quantities to that type -- the factors, every
    intermediate of S^T lambda, mu, M^T mu and lambda after each update --
    to model what a lower-precision evaluation of the same recursion loses
    (the arithmetic itself stays FP64).
    """
    diff = list(workload.diff if diff is None else diff)
    params = tuple(workload.params if params is None else params)
    n = tuple(workload.n if n is None else n)
    se = SplitEE(workload.geometry, n, diff, workload.tau, workload.extent)
    react = lambda U: reactions.reaction(workload.reaction, U, params)  # noqa: E731
    # forward, storing all states (oracle sizes are small)
    states = [list(W0s)]
    for _ in range(steps):
        states.append(se.step(states[-1], react, w_dirichlet=w_dirichlet))
    resid = states[-1][0] - target
    L = 0.5 * float(np.sum(resid * resid))
    lam = [resid] + [np.zeros_like(W) for W in W0s[1:]]
    ns = len(W0s)
    ops = [chain(se, s) for s in range(ns)]
    rnd = None
    if round_to is not None:
        rnd = lambda X: np.asarray(X).astype(round_to).astype(np.float64)  # noqa: E731
        ops = [[(o[0], rnd(o[1])) + tuple(o[2:]) for o in chain_s] for chain_s in ops]
        lam = [rnd(x) for x in lam]
    g_d = np.zeros(ns)
    g_p = np.zeros(len(params))
    Mt = se.M.T.tocsr()
    for it in range(steps - 1, -1, -1):
        Ws = states[it]
        G = react(Ws)
        J = reactions.jacobian(workload.reaction, Ws, params)
        dGp = param_derivative(workload.reaction, Ws, params)
        mus = [se.tau * apply_chain_T(ops[s], lam[s], rnd) for s in range(ns)]
        if rnd is not None:
            mus = [rnd(m) for m in mus]
        new = []
        for s in range(ns):
            wd = 0.0 if w_dirichlet is None else w_dirichlet[s]
            MW = assemble.unvec(se.M @ assemble.vec(Ws[s]) + se.lift * wd, n)
            F = diff[s] * MW + G[s]
            g_d[s] += se.tau * float(np.sum(lam[s] * apply_chain_dd(ops[s], F)))
            g_d[s] += float(np.sum(mus[s] * MW))
            MtMu = assemble.unvec(Mt @ assemble.vec(mus[s]), n)
            if rnd is not None:
                MtMu = rnd(diff[s] * MtMu) / diff[s]
            acc = lam[s] + diff[s] * MtMu
            for r in range(ns):
                acc = acc + J[r][s] * mus[r]
            new.append(acc if rnd is None else rnd(acc))
        for r in range(ns):
            for q in range(len(params)):
                g_p[q] += float(np.sum(mus[r] * dGp[r][q]))
        lam = new
    return L, lam, g_d, g_p


def loss(workload, W0s, target, steps, n=None, diff=None, params=None, w_dirichlet=None):
    diff = list(workload.diff if diff is None else diff)
    params = tuple(workload.params if params is None else params)
    n = tuple(workload.n if n is None else n)
    se = SplitEE(workload.geometry, n, diff, workload.tau, workload.extent)
    react = lambda U: reactions.reaction(workload.reaction, U, params)  # noqa: E731
    Ws = list(W0s)
    for _ in range(steps):
        Ws = se.step(Ws, react, w_dirichlet=w_dirichlet)
    r = Ws[0] - target
    return 0.5 * float(np.sum(r * r))
