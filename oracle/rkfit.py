"""Shared-pole rational approximants of exp(-t x) on x >= 0 by RKFIT.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.2, eq. (ratfam): one denominator for all channels t_1..t_K,
    r^[j](x) = sum_i alpha_i^[j] / (x - xi_i)  ~  exp(-t_j x),  x >= 0,
of subdiagonal type [(m-1)/m] (no constant term).  The poles come from
RKFIT (Berljafa & Guettel, cited in Sec. 3.2), which approximately minimizes
eq. (rkfit), sum_j w_j || r^[j](S) v - exp(-t_j S) v ||^2, for a diagonal
surrogate S with dense eigenvalues on [0, inf) and v = ones, by implicit pole
relocation.  Each sweep:

  1. builds an orthonormal basis V of the rational Krylov space
     Q_{m+1}(S, v, q_m) with the current poles by the rational Arnoldi
     method, which also yields the pencil (H, K) with S V K = V H;
  2. finds the unit vector c minimizing sum_j w_j ||(I - V V^*) F_j V c||^2,
     F_j = exp(-t_j S) (right singular vector of the stacked matrix for its
     smallest singular value);
  3. takes as new poles the roots of the rational function represented by
     V c, i.e. the eigenvalues of the trailing m x m part of the pencil
     (Q^* H, Q^* K), Q unitary with first column c.

Readings of passages the paper leaves open (listed in the design notes):
  * eq. (rkfit) is printed with exp(t S) and without the channel index; it is
    read as exp(-t_j S) v with the weight w_j on channel j's squared norm;
  * the surrogate S: x = 0 and 2000 log-spaced points on [1e-3, 1e4/tau_min]
    in the normalized time tau = t/t_max (see ``surrogate``);
  * initial poles: m/2 conjugate pairs -r(cos 60deg +- i sin 60deg), r
    log-spaced on [1, 1/tau_min] (plus -1/sqrt(tau_min) for odd m); 20 sweeps,
    keeping the sweep whose fit has the smallest uniform error of eq.
    (uniform_error), max_j w_j max_x |exp(-t_j x) - r^[j](x)|, on the samples;
  * the relocated poles are symmetrized into conjugate pairs; poles may lie in
    either half plane (Sec. 3.3 only asks that they avoid the spectral region
    x >= 0), and a real pole on x >= 0 is reflected to -x;
  * after the last sweep the residues of every channel are the least-squares
    fit over the subdiagonal basis {1/(x - xi_i)} on the samples, in real
    arithmetic with (Re, Im) pairs, so conjugate symmetry holds exactly;
  * time scaling: exp(-t x) = exp(-tau (t_max x)), so poles and residues
    fitted in tau are divided by t_max.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

HALPHEN = 9.289025491920818  # Halphen's constant H (Sec. 3.3)


def surrogate(tau_min: float, ns: int = 2000) -> np.ndarray:
    """Eigenvalues of the diagonal surrogate S: 0 and ns log-spaced points."""
    return np.concatenate([[0.0], np.logspace(-3.0, np.log10(1e4 / tau_min), ns)])


def initial_poles(m: int, tau_min: float) -> np.ndarray:
    r = np.logspace(0.0, np.log10(1.0 / tau_min), m // 2)
    th = np.pi / 3
    xi = np.concatenate([-r * np.exp(1j * th), -r * np.exp(-1j * th)])
    if m % 2:
        xi = np.concatenate([xi, [-1.0 / np.sqrt(tau_min)]])
    return xi


def rational_arnoldi(s: np.ndarray, v: np.ndarray, xi: np.ndarray):
    """Orthonormal V (N x m+1) and (m+1) x m pencil (H, K) with S V K = V H.

    Step j solves (S - xi_j I) w = v_j (S diagonal), orthogonalizes w against
    v_1..v_j twice (classical Gram-Schmidt) and normalizes; with coefficients
    k = [h; beta] this gives (S - xi_j) V_{j+1} k = v_j, i.e. column j of
    K is k and column j of H is xi_j k + e_j.
    """
    n, m = len(s), len(xi)
    V = np.zeros((n, m + 1), complex)
    K = np.zeros((m + 1, m), complex)
    H = np.zeros((m + 1, m), complex)
    V[:, 0] = v / np.linalg.norm(v)
    for j in range(m):
        w = V[:, j] / (s - xi[j])
        k = np.zeros(j + 2, complex)
        for _ in range(2):
            h = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ h
            k[:j + 1] += h
        k[j + 1] = np.linalg.norm(w)
        V[:, j + 1] = w / k[j + 1]
        K[:j + 2, j] = k
        H[:j + 2, j] = xi[j] * k
        H[j, j] += 1.0
    return V, K, H


def relocate(V, K, H, F, w):
    """One RKFIT pole relocation; returns (new poles, misfit)."""
    blocks = []
    for wj, Fj in zip(w, F):
        FV = Fj[:, None] * V
        blocks.append(np.sqrt(wj) * (FV - V @ (V.conj().T @ FV)))
    R = np.linalg.qr(np.vstack(blocks), mode="r")
    _, sv, Vh = np.linalg.svd(R)
    c = Vh[-1].conj()
    # unitary Q whose first column is c
    Q, _ = np.linalg.qr(np.column_stack([c, np.eye(len(c))[:, 1:]]))
    Q[:, 0] = c  # QR may flip its sign/phase; the span is what matters
    Ht = Q.conj().T @ H
    Kt = Q.conj().T @ K
    z = sla.eigvals(Ht[1:], Kt[1:])
    return z, sv[-1]


def symmetrize(z: np.ndarray, prev: np.ndarray, rel: float = 1e-10) -> np.ndarray:
    """Conjugate-pair symmetrization of relocated poles (real input data gives
    a real rational function, so poles come in conjugate pairs up to rounding)."""
    z = np.asarray(z, complex)
    bad = ~np.isfinite(z)
    if bad.any():  # roots at infinity: keep the previous poles in their place
        z[bad] = prev[np.argsort(-np.abs(prev))[:bad.sum()]]
    near = np.abs(z.imag) <= rel * np.abs(z)
    reals = list(z[near].real)
    up = list(z[~near & (z.imag > 0)])
    lo = list(z[~near & (z.imag < 0)].conj())
    out = []
    while up and lo:
        d = np.abs(np.subtract.outer(np.array(up), np.array(lo)))
        a, b = np.unravel_index(np.argmin(d), d.shape)
        p = 0.5 * (up.pop(a) + lo.pop(b))
        out += [p, p.conjugate()]
    reals += [u.real for u in up] + [u.real for u in lo]
    reals = [-abs(r) if r >= 0 else r for r in reals]  # no pole on x >= 0
    return np.array(out + [complex(r) for r in reals])


def representatives(poles: np.ndarray) -> np.ndarray:
    """One pole per conjugate pair (Im > 0), followed by the real poles."""
    poles = np.asarray(poles, complex)
    up = poles[poles.imag > 0]
    re = poles[poles.imag == 0]
    return np.concatenate([up[np.argsort(np.abs(up))], re[np.argsort(np.abs(re))]])


def fit_residues(reps: np.ndarray, tau: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Least-squares residues for every channel (no constant term, eq. (ratfam)).

    Returns A (J x K complex): r^[k](x) = sum_j 2 Re(A_jk/(x - p_j)) over the
    pair representatives plus sum_j A_jk/(x - p_j) over real poles.
    """
    cols = []
    for p in reps:
        g = 1.0 / (x - p)
        cols += [2 * g.real, -2 * g.imag] if p.imag > 0 else [g.real]
    B = np.column_stack(cols)
    scale = np.linalg.norm(B, axis=0)
    Y = np.exp(-np.outer(x, tau))
    coef = np.linalg.lstsq(B / scale, Y, rcond=1e-30)[0] / scale[:, None]
    A = np.zeros((len(reps), len(tau)), complex)
    r = 0
    for jj, p in enumerate(reps):
        if p.imag > 0:
            A[jj] = coef[r] + 1j * coef[r + 1]
            r += 2
        else:
            A[jj] = coef[r]
            r += 1
    return A


def evaluate(reps: np.ndarray, A: np.ndarray, x: np.ndarray) -> np.ndarray:
    """r^[k](x) for all channels k (len(x) x K), real-valued."""
    out = np.zeros((len(x), A.shape[1]))
    for jj, p in enumerate(reps):
        g = 1.0 / (x - p)
        term = np.outer(g, A[jj])
        out += 2 * term.real if p.imag > 0 else term.real
    return out


def check_points(tau_min: float, n: int = 200000) -> np.ndarray:
    """Dense x >= 0 set for the uniform error: 0 and log-spaced points far past
    the point where exp(-tau_min x) underflows."""
    return np.concatenate([[0.0], np.logspace(-6.0, np.log10(1e8 / tau_min), n)])


def channel_errors(reps, A, tau, x=None, chunk=20000) -> np.ndarray:
    """eq. (error): max_{x>=0} |exp(-t_j x) - r^[j](x)| per channel, on the
    dense check set; beyond its last point the error is |sum of residues|/x up
    to O(1/x^2), which is added as a bound."""
    if x is None:
        x = check_points(float(np.min(tau)))
    err = np.zeros(len(tau))
    for s in range(0, len(x), chunk):
        xs = x[s:s + chunk]
        e = np.abs(np.exp(-np.outer(xs, tau)) - evaluate(reps, A, xs)).max(axis=0)
        err = np.maximum(err, e)
    # beyond the last point x_max (far past every pole) r(x) ~ (sum of residues)/x
    lead = np.zeros(len(tau))
    for jj, p in enumerate(reps):
        lead += 2 * A[jj].real if p.imag > 0 else A[jj].real
    return np.maximum(err, np.abs(lead) / x[-1])


def rkfit(t, degree: int, w=None, sweeps: int = 20, ns: int = 2000):
    """Shared poles and residues for channels t (any positive times).

    Returns a dict with
      xi     poles xi_i of eq. (ratfam) in physical units (one per pair + reals),
      alpha  residues alpha_i^[k] (J x K), so that
             r^[k](x) = sum over pairs 2 Re(alpha/(x - xi)) + sum over reals,
      err    eq. (error) per channel,
      degree the number of poles m-hat.
    """
    t = np.asarray(t, float)
    if np.any(~np.isfinite(t)) or np.any(t <= 0):
        raise ValueError("channel times must be positive and finite")
    if w is None:
        w = np.ones(len(t))
    tmax = t.max()
    tau = t / tmax
    s = surrogate(tau.min(), ns)
    v = np.ones_like(s)
    F = np.exp(-np.outer(tau, s))
    poles = initial_poles(degree, tau.min())
    xsel = check_points(tau.min(), 4000)  # coarse uniform-error proxy for sweep selection
    best = None
    for _ in range(sweeps):
        V, K, H = rational_arnoldi(s, v, poles)
        z, _mis = relocate(V, K, H, F, w)
        poles = symmetrize(z, poles)
        reps = representatives(poles)
        A = fit_residues(reps, tau, s)
        e = (w * channel_errors(reps, A, tau, xsel)).max()   # eq. (uniform_error), weighted
        if best is None or e < best[0]:
            best = (e, reps, A)
    _, reps, A = best
    err = channel_errors(reps, A, tau)
    return {"xi": reps / tmax, "alpha": A / tmax, "err": err, "degree": degree,
            "pairs": reps.imag > 0}


def shifts_and_coefficients(fit: dict):
    """Convert to the solver's form: shifts s_j = -xi_j for (K + s_j M) x_j = f
    and contraction coefficients c_j(t_k) = 2 alpha_j^[k] (pair) or alpha_j^[k]
    (real pole), so that u(t_k) = Re sum_j c_j(t_k) x_j (eq. (rmj))."""
    xi = fit["xi"]
    c = np.where(fit["pairs"][:, None], 2.0, 1.0) * fit["alpha"]
    return -xi, c


# -- degree arithmetic of Sec. 3.3 and Table 1 -------------------------------

def single_time_degree(tol: float) -> int:
    """Smallest m with 2 H^(-m-1/2) <= tol (the asymptotic best-approximation
    error of exp(-x) of type [m/m], Sec. 3.3)."""
    m = 0
    while 2.0 * HALPHEN ** (-m - 0.5) > tol:
        m += 1
    return m


def break_even(m_hat: int, m: int) -> float:
    """K* = ceil(m_hat/2) / ceil(m/2) (Sec. 3.3)."""
    return -(-m_hat // 2) / -(-m // 2)


def solve_counts(m: int, K: int, m_hat: int):
    """Shifted solves: K*ceil(m/2) for single-time approximants, ceil(m_hat/2)
    for the shared-pole family (Sec. 3.1, 3.2)."""
    return K * -(-m // 2), -(-m_hat // 2)
