"""Gauss-Newton inversion for ln sigma with CGLS on the Jacobian actions
(Sec. 4: "Using iterative solvers" and "Regularization").

The Jacobian J of the receiver data with respect to m = ln sigma is never
formed.  CGLS needs only the actions J x (tem_jacobian_apply) and J^T y
(tem_adjoint: the gradient of y^T d), each one set of shifted solves on the
device.  Tikhonov regularization towards a reference model m_r appends
sqrt(lam) I to J and sqrt(lam) (m_r - m) to the right-hand side.  Only the
cells in `active` (the earth) are parameters; the air stays fixed.

`cgls` is written against plain callables so that it can run on any pair of
actions; `gauss_newton_step` drives it with the library's.
"""
from __future__ import annotations

import numpy as np


def cgls(jvp, vjp, b, n, lam=0.0, c=None, iters=10, tol=0.0):
    """Least-squares solution x of min ||J x - b||^2 + lam ||x - c||^2 by CGLS
    (conjugate gradients on the normal equations, in the product form that
    applies J and J^T once per iteration).  jvp(x) -> J x (flat), vjp(y) -> J^T y
    (flat); b has the length of the data, x and c the number of parameters n.
    Returns (x, history of the residual norms of the normal equations)."""
    b = np.asarray(b, float).ravel()
    c = np.zeros(n) if c is None else np.asarray(c, float).ravel()
    sl = np.sqrt(lam)
    x = np.zeros(n)
    # augmented residual [b - J x; sl (c - x)] and s = A^T r
    rd, rm = b.copy(), sl * c
    s = vjp(rd) + sl * rm
    p = s.copy()
    gamma = float(s @ s)
    hist = [np.sqrt(gamma)]
    for _ in range(iters):
        if gamma == 0.0 or (tol > 0.0 and np.sqrt(gamma) <= tol * hist[0]):
            break
        qd, qm = jvp(p), sl * p
        alpha = gamma / float(qd @ qd + qm @ qm)
        x += alpha * p
        rd -= alpha * qd
        rm -= alpha * qm
        s = vjp(rd) + sl * rm
        gamma_new = float(s @ s)
        hist.append(np.sqrt(gamma_new))
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
    return x, hist


def misfit(d, d_obs, wd, m, m_ref, lam):
    """phi = 1/2 ||wd (d - d_obs)||^2 + lam/2 ||m - m_ref||^2 (m over the active cells)."""
    r = (wd * (d - d_obs)).ravel()
    return 0.5 * float(r @ r) + 0.5 * lam * float(np.sum((m - m_ref) ** 2))


def gauss_newton_step(ctx, wl, xi, c, d_obs, active, m_ref=None, lam=0.0, wd=None, cgls_iters=5,
                      steps=(1.0, 0.5, 0.25, 0.125)):
    """One Gauss-Newton step (Sec. 4) from the conductivity currently set on
    ctx (taken from wl.sigma): forward with kept solutions, CGLS on
    [wd J; sqrt(lam) I] dm = [-wd r; sqrt(lam)(m_ref - m)] over the active cells,
    then the first step length in `steps` that lowers the misfit.  The context
    ends with the accepted model set.  Returns (new sigma, info)."""
    sigma = np.asarray(wl.sigma, float)
    m_full = np.log(sigma)
    m = m_full[active]
    m_ref = m.copy() if m_ref is None else np.asarray(m_ref, float)
    ctx.set_conductivity(sigma)
    d, _ = ctx.forward(wl.loops, wl.receivers, xi, c, keep_solutions=True)
    wd = np.ones_like(d) if wd is None else np.asarray(wd, float)
    phi0 = misfit(d, d_obs, wd, m, m_ref, lam)

    def jvp(x):
        dm = np.zeros(sigma.shape)
        dm[active] = x
        dd, _ = ctx.jacobian_apply(dm)
        return (wd * dd).ravel()

    def vjp(y):
        g, _ = ctx.adjoint(wd * np.asarray(y).reshape(d.shape))
        return g[active]

    b = -(wd * (d - d_obs)).ravel()
    dm, hist = cgls(jvp, vjp, b, int(np.count_nonzero(active)), lam=lam, c=m_ref - m, iters=cgls_iters)
    info = {"phi0": phi0, "cgls_normal_residuals": hist, "tried": []}
    for a in steps:
        m_new = m_full.copy()
        m_new[active] = m + a * dm
        sig_new = np.exp(m_new)
        ctx.set_conductivity(sig_new)
        dn, _ = ctx.forward(wl.loops, wl.receivers, xi, c)
        phi = misfit(dn, d_obs, wd, m_new[active], m_ref, lam)
        info["tried"].append((a, phi))
        if phi < phi0:
            info.update(step=a, phi=phi)
            return sig_new, info
    ctx.set_conductivity(sigma)
    info.update(step=0.0, phi=phi0)
    return sigma, info
