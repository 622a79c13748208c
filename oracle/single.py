"""Single-time rational best approximation of exp(-x) on [0, inf) and its
evaluation by direct shifted solves (Sec. 3.1, eq. (rba)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The approximant is the type-[m/m] rational function in partial fractions,
    r_m(x) = alpha_0 + sum_{i=1}^m alpha_i / (x - xi_i)  ~  exp(-x),  x >= 0,
and for one time t
    exp(-t M^-1 K) b ~ r_m(t M^-1 K) b = alpha_0 b + sum_i alpha_i (t K - xi_i M)^-1 f,
with b = M^-1 f.  Every channel t_k has its own shifted matrices t_k K - xi_i M,
so K channels cost K ceil(m/2) solves (conjugate poles share one solve).

Readings of passages the paper leaves open (listed in the design notes):
  * the paper takes the best uniform approximation (Cody, Meinardus and Varga;
    Trefethen's ATAP, ch. 25) without saying how it is computed.  Here it is
    computed by RKFIT pole relocation (the machinery of ``rkfit``) on the one
    channel t = 1 with a constant term, followed by Lawson's iteratively
    reweighted least squares, which drives the least-squares fit to the
    minimax one: after 5 unweighted sweeps, each sweep multiplies the sample
    weights by |error|^(1/2) (normalized to max 1) and relocates the poles in
    the weighted inner product (starting vector sqrt(w)).  The sweep with the
    smallest uniform error is kept.  The result equioscillates at 2m + 2
    points to within a few per mille, so by de la Vallee Poussin's theorem
    its error is within that much of the best (checked by the pins);
  * samples: x = 0 and x = 9 (1 + s)/(1 - s) at 2000 Chebyshev points
    s = -cos(theta) in [-1, 1) (the map of [0, inf) to [-1, 1) with the
    scale 9 used for this function by Trefethen, Weideman and Schmelzer);
  * the uniform error is measured on 0, log-spaced points to 1e8 and at
    x = infinity, where r_m equals alpha_0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import rkfit as _rk


def samples(n: int = 2000, scale: float = 9.0) -> np.ndarray:
    """x = 0 and x = scale (1 + s)/(1 - s) at Chebyshev points s in [-1, 1)."""
    th = np.linspace(0.0, np.pi, n)[1:]
    s = -np.cos(th)
    s = s[s < 1.0]
    return np.concatenate([[0.0], scale * (1.0 + s) / (1.0 - s)])


def _basis(reps: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Real basis of type-[m/m] functions with the poles reps: the constant,
    then (2 Re g, -2 Im g) per conjugate pair and Re g per real pole,
    g = 1/(x - p)."""
    cols = [np.ones_like(x)]
    for p in reps:
        g = 1.0 / (x - p)
        cols += [2 * g.real, -2 * g.imag] if p.imag > 0 else [g.real]
    return np.column_stack(cols)


def fit_with_constant(reps: np.ndarray, x: np.ndarray, w=None):
    """Weighted least-squares alpha_0 and residues for exp(-x) with the poles
    reps: minimizes sum_l w_l |exp(-x_l) - r(x_l)|^2.  Returns (alpha0,
    alpha[J] complex) in the form r(x) = alpha0 + sum over pairs
    2 Re(alpha/(x - p)) + sum over real poles alpha/(x - p)."""
    B = _basis(reps, x)
    y = np.exp(-x)
    if w is not None:
        sw = np.sqrt(w)
        B, y = B * sw[:, None], y * sw
    scale = np.linalg.norm(B, axis=0)
    coef = np.linalg.lstsq(B / scale, y, rcond=1e-30)[0] / scale
    alpha = np.zeros(len(reps), complex)
    r = 1
    for jj, p in enumerate(reps):
        if p.imag > 0:
            alpha[jj] = coef[r] + 1j * coef[r + 1]
            r += 2
        else:
            alpha[jj] = coef[r]
            r += 1
    return float(coef[0]), alpha


def evaluate(fit: dict, x: np.ndarray) -> np.ndarray:
    """r_m(x) for real x (the conjugate partner of each pair included)."""
    x = np.asarray(x, float)
    out = np.full(x.shape, fit["alpha0"])
    for p, a in zip(fit["xi"], fit["alpha"]):
        g = a / (x - p)
        out = out + (2 * g.real if p.imag > 0 else g.real)
    return out


def uniform_error(fit: dict, x=None, chunk: int = 50000) -> float:
    """max_{x >= 0} |exp(-x) - r_m(x)| on a dense check set and at infinity."""
    if x is None:
        x = np.concatenate([[0.0], np.logspace(-6.0, 8.0, 200000)])
    e = abs(fit["alpha0"])
    for s in range(0, len(x), chunk):
        xs = x[s:s + chunk]
        e = max(e, float(np.abs(np.exp(-xs) - evaluate(fit, xs)).max()))
    return e


def best_rational(m: int, sweeps: int = 80, unweighted: int = 5, n: int = 2000) -> dict:
    """Type-[m/m] best uniform approximation of exp(-x) on [0, inf).

    Returns a dict with xi (one pole per conjugate pair with Im > 0, then the
    real poles), alpha (their residues), alpha0, pairs (bool per pole), err
    (the uniform error) and m."""
    if m < 1:
        raise ValueError("degree must be at least 1")
    x = samples(n)
    y = np.exp(-x)
    w = np.ones_like(x)
    poles = _rk.initial_poles(m, 1.0)
    best = None
    for sweep in range(sweeps):
        V, K, H = _rk.rational_arnoldi(x, np.sqrt(w), poles)
        z, _ = _rk.relocate(V, K, H, [y], [1.0])
        poles = _rk.symmetrize(z, poles)
        reps = _rk.representatives(poles)
        a0, alpha = fit_with_constant(reps, x, w)
        fit = {"xi": reps, "alpha": alpha, "alpha0": a0}
        err = uniform_error(fit, np.concatenate([[0.0], np.logspace(-6.0, 8.0, 4000)]))
        if best is None or err < best[0]:
            best = (err, fit)
        if sweep + 1 >= unweighted:
            e = np.abs(y - evaluate(fit, x))
            w = w * np.sqrt(e)
            w = np.maximum(w / w.max(), 1e-300)
    fit = best[1]
    fit["pairs"] = fit["xi"].imag > 0
    fit["err"] = uniform_error(fit)
    fit["m"] = m
    return fit


def alternation(fit: dict, x=None):
    """Signed extremal values of the error e(x) = exp(-x) - r_m(x) that
    alternate in sign, in increasing x (with x = infinity, where e = -alpha0,
    appended last): on each maximal run of one sign the extremum of |e|."""
    if x is None:
        x = np.concatenate([[0.0], np.logspace(-8.0, 8.0, 400000)])
    e = np.exp(-x) - evaluate(fit, x)
    e = np.concatenate([e, [-fit["alpha0"]]])
    ext = []
    sign = 0
    for v in e:
        s = 1 if v > 0 else (-1 if v < 0 else 0)
        if s == 0:
            continue
        if s != sign:
            ext.append(v)
            sign = s
        elif abs(v) > abs(ext[-1]):
            ext[-1] = v
    return np.array(ext)


def shifted_solve(prob, t: float, xi: complex, f: np.ndarray) -> np.ndarray:
    """x = (t K - xi M)^-1 f by a sparse LU of the matrix as written."""
    A = (t * prob.K - xi * sp.diags(prob.M)).astype(complex).tocsc()
    return spla.splu(A, permc_spec="MMD_AT_PLUS_A").solve(np.asarray(f, complex))


def forward_single(prob, fit: dict, t, src: int = 0, terms: bool = False):
    """eq. (rba) for every channel t_k: u(t_k) = alpha_0 b + sum_i alpha_i
    (t_k K - xi_i M)^-1 f, the conjugate pole of a pair contributing the
    conjugate term (so the pair gives 2 Re).  Returns the fields U (n x K) and
    the receiver data d (K x n_rx); with terms, also S (K): the sum of the
    M-norms of the terms, S_k = |alpha_0| ||b||_M + sum_i |alpha_i|
    ||(t_k K - xi_i M)^-1 f||_M over all m poles (the scale of the rounding
    in the sum)."""
    f = prob.F[:, src]
    b = f / prob.M
    t = np.atleast_1d(np.asarray(t, float))
    U = np.zeros((len(f), len(t)))
    S = np.zeros(len(t))
    mn = lambda v: float(np.sqrt(np.sum(prob.M * np.abs(v) ** 2)))
    for k, tk in enumerate(t):
        u = fit["alpha0"] * b
        S[k] = abs(fit["alpha0"]) * mn(b)
        for p, a, pair in zip(fit["xi"], fit["alpha"], fit["pairs"]):
            x = shifted_solve(prob, tk, p, f)
            term = a * x
            u = u + (2 * term.real if pair else term.real)
            S[k] += (2 if pair else 1) * abs(a) * mn(x)
        U[:, k] = u
    if terms:
        return U, (prob.Q @ U).T, S
    return U, (prob.Q @ U).T


def solves(fit: dict, K: int) -> int:
    """Shifted systems eq. (rba) needs for K channels: one per pole
    representative (a conjugate pair shares one) per channel."""
    return K * len(fit["xi"])
