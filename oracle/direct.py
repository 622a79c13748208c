"""Shifted solves, residue contraction, receiver data, dense references and
the adjoint gradient -- all by direct methods in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Forward (Sec. 3.2, eq. (rmj) and the S R product that follows it): for the
shared poles xi_i and residues alpha_i^[k],
    u(t_k) ~ r^[k](M^-1 K) b = sum_i alpha_i^[k] (K - xi_i M)^-1 f,
evaluated as U = Re(X C) with X = [x_1 .. x_J], x_j = (K + s_j M)^-1 f,
s_j = -xi_j (one system per conjugate pair, plus one per real pole) and
c_j(t_k) = 2 alpha_j^[k] for a pair, alpha_j^[k] for a real pole.  Receiver
data are d_k = Q u(t_k) (Sec. 5).

Each x_j is the plain definition: a pivoted LU solve of the shifted matrix,
by a banded LU after reverse Cuthill-McKee ordering (LAPACK gbsv) or by a
general sparse LU (SuperLU) as an independent second solver.

Jacobian action and adjoint (Sec. 4): with M(m) = sum_c e^{m_c} M_c,
dA_j/dm_c = s_j e^{m_c} M_c.  The action J dm solves A_j dx_j = -(dA_j dm) x_j
and contracts the dx_j like the forward; the adjoint (J^T w) of a misfit
phi(d) with w = dphi/dd is
    dphi/dm_c = -Re sum_j s_j (lambda_j^T  e^{m_c} M_c  x_j),
    lambda_j  = A_j^-T g_j = A_j^-1 g_j   (A_j complex symmetric),
    g_j       = sum_k c_j(t_k) Q^T w_k.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import reverse_cuthill_mckee


def _shifted(K, M, s):
    return (K + sp.diags(s * M)).astype(complex)


class BandedSolver:
    """Pivoted banded LU of K + s M after a reverse Cuthill-McKee ordering."""

    def __init__(self, K):
        self.perm = reverse_cuthill_mckee(sp.csr_matrix(K), symmetric_mode=True)
        Kp = sp.csr_matrix(K)[self.perm][:, self.perm].tocoo()
        self.bw = int(np.max(np.abs(Kp.row - Kp.col))) if Kp.nnz else 0
        self.Kp = Kp

    def solve(self, M, s, rhs):
        n = self.Kp.shape[0]
        p, bw = self.perm, self.bw
        A = (self.Kp + sp.diags(s * M[p])).tocoo()
        ab = np.zeros((2 * bw + 1, n), complex)
        ab[bw + A.row - A.col, A.col] = A.data
        x = sla.solve_banded((bw, bw), ab, np.asarray(rhs, complex)[p], check_finite=False)
        out = np.empty_like(x)
        out[p] = x
        return out


def solve_shifted(prob, shifts, rhs=None, method="splu"):
    """X (n x J [x n_src]) with (K + s_j M) X[:, j] = rhs (default: the loop sources)."""
    rhs = prob.F if rhs is None else rhs
    rhs = np.asarray(rhs)
    single = rhs.ndim == 1
    R = rhs[:, None] if single else rhs
    X = np.zeros((R.shape[0], len(shifts), R.shape[1]), complex)
    banded = BandedSolver(prob.K) if method == "banded" else None
    for j, s in enumerate(shifts):
        if method == "banded":
            for c in range(R.shape[1]):
                X[:, j, c] = banded.solve(prob.M, s, R[:, c])
        else:
            lu = spla.splu(_shifted(prob.K, prob.M, s).tocsc(), permc_spec="MMD_AT_PLUS_A")
            X[:, j, :] = lu.solve(R.astype(complex))
    return X[:, :, 0] if single else X


def contract(X, C):
    """U = Re(X C): all channels at once (the S R product of Sec. 3.2)."""
    return (X @ C).real


def forward(prob, shifts, C, method="splu"):
    """Per source: X (n x J), fields U (n x T) and receiver data d (T x n_rx)."""
    out = []
    for src in range(prob.F.shape[1]):
        X = solve_shifted(prob, shifts, prob.F[:, src], method)
        U = contract(X, C)
        d = (prob.Q @ U).T
        out.append({"X": X, "U": U, "d": d})
    return out


def m_norm(prob, v):
    """||v||_M = (v^T M v)^(1/2) column-wise (Sec. 3.3)."""
    v = np.asarray(v)
    if v.ndim == 1:
        return float(np.sqrt(np.sum(prob.M * np.abs(v) ** 2)))
    return np.sqrt(np.einsum("n,nk->k", prob.M, np.abs(v) ** 2))


def dense_exact(prob, t, src=0):
    """u(t) = exp(-t M^-1 K) b, b = M^-1 f (eq. (expm)) from the eigen-
    decomposition of the symmetric M^-1/2 K M^-1/2 (tiny grids only)."""
    Dm = 1.0 / np.sqrt(prob.M)
    A = (Dm[:, None] * prob.K.toarray()) * Dm[None, :]
    lam, V = np.linalg.eigh(A)
    lam = np.maximum(lam, 0.0)
    b = prob.F[:, src] / prob.M
    y0 = V.T @ (np.sqrt(prob.M) * b)
    return np.stack([Dm * (V @ (np.exp(-tk * lam) * y0)) for tk in np.atleast_1d(t)], axis=1)


def dense_expm(prob, t, src=0):
    """The same quantity by scipy's Pade-based expm of -t M^-1 K."""
    B = -(prob.K.toarray() / prob.M[:, None])
    b = prob.F[:, src] / prob.M
    return np.stack([sla.expm(tk * B) @ b for tk in np.atleast_1d(t)], axis=1)


def misfit_gradient(prob, shifts, C, w, X=None, method="splu"):
    """Gradient of phi w.r.t. ln sigma per cell, given w = dphi/dd (T x n_rx)
    for source 0, by the adjoint formula of Sec. 4."""
    if X is None:
        X = solve_shifted(prob, shifts, prob.F[:, 0], method)
    G = prob.Q.T @ np.asarray(w).T          # n x T: Q^T w_k
    Gj = G @ C.T                             # n x J: g_j = sum_k c_jk Q^T w_k
    Lam = np.zeros_like(X)
    for j, s in enumerate(shifts):
        Lam[:, j] = solve_shifted(prob, [s], Gj[:, j], method)[:, 0]
    D = prob.mass_derivative()               # n x cells: dM/d ln sigma
    grad = np.zeros(D.shape[1])
    for j, s in enumerate(shifts):
        grad -= (s * (D.T @ (Lam[:, j] * X[:, j]))).real
    return grad


def jacobian_apply(prob, shifts, C, dm, X=None, method="splu"):
    """J dm: the first-order change of the receiver data (T x n_rx, source 0)
    for a change dm of ln sigma per cell (Sec. 4, eq. (rmjQ) differentiated):
    A_j dx_j = -(dA_j/dm . dm) x_j = -s_j (dM/d ln sigma . dm) x_j, and
    dd_k = Q Re sum_j c_jk dx_j."""
    if X is None:
        X = solve_shifted(prob, shifts, prob.F[:, 0], method)
    dM = prob.mass_derivative() @ np.asarray(dm)   # per edge
    dX = np.zeros_like(X)
    for j, s in enumerate(shifts):
        dX[:, j] = -solve_shifted(prob, [s], s * dM * X[:, j], method)[:, 0]
    return (prob.Q @ contract(dX, C)).T


def data_for_model(prob_factory, sigma, shifts, C, method="splu"):
    """Receiver data (T x n_rx) of source 0 for conductivity sigma."""
    prob = prob_factory(sigma)
    X = solve_shifted(prob, shifts, prob.F[:, 0], method)
    return (prob.Q @ contract(X, C)).T
