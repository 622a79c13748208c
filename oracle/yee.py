"""Explicit Yee-grid (lowest-order edge element, lumped mass) operators.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper discretizes eq. (pde) with Nedelec edge elements and obtains the
semi-discrete system eq. (ode), K u + M u' = 0, M u(0) = f, with
K_ij = (mu^-1 curl Phi_j, curl Phi_i), M_ij = (sigma Phi_j, Phi_i) and
f_i = (q, Phi_i) (Sec. 2.2).  Here the same three objects are formed on a
tensor grid of hexahedra with one unknown per edge (the tangential field at
the edge midpoint):

  * K = C^T W C, where row f of C is the circulation of the edge field around
    face f (edge length times edge value, right-hand orientation) and
    W = diag(h_dual / (mu0 * area)) weights each face by its dual length over
    mu0 and its area, so that e^T K e is the discrete magnetic energy
    sum_f (1/mu0) (c_f/A_f)^2 A_f h_dual_f;
  * M is diagonal with M_e = 1/4 sum over the four cells touching edge e of
    sigma_c V_c (the lumped L2 mass of sigma);
  * f_e = I * l_e * s_e for the edges of the transmitter loop (s_e = +-1 for
    the loop direction against the edge direction), 0 elsewhere;
  * edges in the boundary planes are eliminated (n x e = 0, eq. (bc)).

Edge numbering ("storage" order, also used at the C-ABI for field output):
Ex[Nz+1][Ny+1][Nx], then Ey[Nz+1][Ny][Nx+1], then Ez[Nz][Ny+1][Nx+1], each x
fastest.  Boundary edges are present in storage order and always zero.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MU0 = 4e-7 * np.pi  # Sec. 2.1


class YeeGrid:
    def __init__(self, hx, hy, hz):
        self.hx = np.asarray(hx, float)
        self.hy = np.asarray(hy, float)
        self.hz = np.asarray(hz, float)
        self.Nx, self.Ny, self.Nz = len(self.hx), len(self.hy), len(self.hz)
        Nx, Ny, Nz = self.Nx, self.Ny, self.Nz
        self.n_ex = (Nz + 1) * (Ny + 1) * Nx
        self.n_ey = (Nz + 1) * Ny * (Nx + 1)
        self.n_ez = Nz * (Ny + 1) * (Nx + 1)
        self.n_edges = self.n_ex + self.n_ey + self.n_ez

    # -- edge indices -------------------------------------------------------
    def ex(self, i, j, k):
        return (np.asarray(k) * (self.Ny + 1) + j) * self.Nx + i

    def ey(self, i, j, k):
        return self.n_ex + (np.asarray(k) * self.Ny + j) * (self.Nx + 1) + i

    def ez(self, i, j, k):
        return self.n_ex + self.n_ey + (np.asarray(k) * (self.Ny + 1) + j) * (self.Nx + 1) + i

    def edge_lengths(self):
        Nx, Ny, Nz = self.Nx, self.Ny, self.Nz
        lx = np.broadcast_to(self.hx[None, None, :], (Nz + 1, Ny + 1, Nx)).ravel()
        ly = np.broadcast_to(self.hy[None, :, None], (Nz + 1, Ny, Nx + 1)).ravel()
        lz = np.broadcast_to(self.hz[:, None, None], (Nz, Ny + 1, Nx + 1)).ravel()
        return np.concatenate([lx, ly, lz])

    def interior(self):
        """Boolean mask over storage edges: True for edges not in a boundary plane."""
        Nx, Ny, Nz = self.Nx, self.Ny, self.Nz
        k, j, i = np.meshgrid(np.arange(Nz + 1), np.arange(Ny + 1), np.arange(Nx), indexing="ij")
        mx = (j > 0) & (j < Ny) & (k > 0) & (k < Nz)
        k, j, i = np.meshgrid(np.arange(Nz + 1), np.arange(Ny), np.arange(Nx + 1), indexing="ij")
        my = (i > 0) & (i < Nx) & (k > 0) & (k < Nz)
        k, j, i = np.meshgrid(np.arange(Nz), np.arange(Ny + 1), np.arange(Nx + 1), indexing="ij")
        mz = (i > 0) & (i < Nx) & (j > 0) & (j < Ny)
        return np.concatenate([mx.ravel(), my.ravel(), mz.ravel()])

    @staticmethod
    def dual_widths(h):
        """Node-centred dual widths: half cells at the ends, averages inside."""
        d = np.empty(len(h) + 1)
        d[0], d[-1] = h[0] / 2, h[-1] / 2
        d[1:-1] = (h[:-1] + h[1:]) / 2
        return d

    # -- operators ------------------------------------------------------------
    def curl(self):
        """(C, w): C maps storage edges to face circulations (lengths included),
        w holds the face weights h_dual/(mu0 A)."""
        hx, hy, hz = self.hx, self.hy, self.hz
        Nx, Ny, Nz = self.Nx, self.Ny, self.Nz
        dx, dy, dz = self.dual_widths(hx), self.dual_widths(hy), self.dual_widths(hz)
        rows, cols, vals, weights = [], [], [], []
        nf = 0
        # faces normal to x: (i in 0..Nx, j < Ny, k < Nz); y -> z -> -y -> -z
        k, j, i = [a.ravel() for a in np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx + 1), indexing="ij")]
        f = nf + np.arange(len(i))
        for e, v in ((self.ey(i, j, k), hy[j]), (self.ez(i, j + 1, k), hz[k]),
                     (self.ey(i, j, k + 1), -hy[j]), (self.ez(i, j, k), -hz[k])):
            rows.append(f); cols.append(e); vals.append(v)
        weights.append(dx[i] / (MU0 * hy[j] * hz[k])); nf += len(i)
        # faces normal to y: (i < Nx, j in 0..Ny, k < Nz); z -> x -> -z -> -x
        k, j, i = [a.ravel() for a in np.meshgrid(np.arange(Nz), np.arange(Ny + 1), np.arange(Nx), indexing="ij")]
        f = nf + np.arange(len(i))
        for e, v in ((self.ez(i, j, k), hz[k]), (self.ex(i, j, k + 1), hx[i]),
                     (self.ez(i + 1, j, k), -hz[k]), (self.ex(i, j, k), -hx[i])):
            rows.append(f); cols.append(e); vals.append(v)
        weights.append(dy[j] / (MU0 * hz[k] * hx[i])); nf += len(i)
        # faces normal to z: (i < Nx, j < Ny, k in 0..Nz); x -> y -> -x -> -y
        k, j, i = [a.ravel() for a in np.meshgrid(np.arange(Nz + 1), np.arange(Ny), np.arange(Nx), indexing="ij")]
        f = nf + np.arange(len(i))
        for e, v in ((self.ex(i, j, k), hx[i]), (self.ey(i + 1, j, k), hy[j]),
                     (self.ex(i, j + 1, k), -hx[i]), (self.ey(i, j, k), -hy[j])):
            rows.append(f); cols.append(e); vals.append(v)
        weights.append(dz[k] / (MU0 * hx[i] * hy[j])); nf += len(i)
        C = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nf, self.n_edges))
        return C, np.concatenate(weights)

    def stiffness_full(self):
        C, w = self.curl()
        return (C.T @ sp.diags(w) @ C).tocsr()

    def gradient(self):
        """G: nodal potential -> edge field (phi_end - phi_start)/l_e, storage edges."""
        Nx, Ny, Nz = self.Nx, self.Ny, self.Nz
        node = lambda i, j, k: (np.asarray(k) * (Ny + 1) + j) * (Nx + 1) + i
        rows, cols, vals = [], [], []
        for comp, shape, step in ((0, (Nz + 1, Ny + 1, Nx), (1, 0, 0)),
                                  (1, (Nz + 1, Ny, Nx + 1), (0, 1, 0)),
                                  (2, (Nz, Ny + 1, Nx + 1), (0, 0, 1))):
            k, j, i = [a.ravel() for a in np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")]
            e = (self.ex, self.ey, self.ez)[comp](i, j, k)
            ell = self.hx[i] if comp == 0 else (self.hy[j] if comp == 1 else self.hz[k])
            a = node(i, j, k)
            b = node(i + step[0], j + step[1], k + step[2])
            rows += [e, e]; cols += [b, a]; vals += [1.0 / ell, -1.0 / ell]
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n_edges, (Nx + 1) * (Ny + 1) * (Nz + 1)))

    def mass_full(self, sigma):
        """Lumped mass on storage edges: M_e = 1/4 sum_{cells c touching e} sigma_c V_c."""
        sigma = np.asarray(sigma, float)
        assert sigma.shape == (self.Nz, self.Ny, self.Nx)
        V = self.hz[:, None, None] * self.hy[None, :, None] * self.hx[None, None, :]
        P = np.zeros((self.Nz + 2, self.Ny + 2, self.Nx + 2))
        P[1:-1, 1:-1, 1:-1] = sigma * V
        # Ex(i,j,k) touches cells (i, j-1..j, k-1..k); P is offset by one
        mx = P[:-1, :-1, 1:-1] + P[:-1, 1:, 1:-1] + P[1:, :-1, 1:-1] + P[1:, 1:, 1:-1]
        my = P[:-1, 1:-1, :-1] + P[:-1, 1:-1, 1:] + P[1:, 1:-1, :-1] + P[1:, 1:-1, 1:]
        mz = P[1:-1, :-1, :-1] + P[1:-1, :-1, 1:] + P[1:-1, 1:, :-1] + P[1:-1, 1:, 1:]
        return 0.25 * np.concatenate([mx.ravel(), my.ravel(), mz.ravel()])

    def mass_derivative_full(self, sigma):
        """Sparse D with D[e, c] = dM_e/d(ln sigma_c) = sigma_c V_c / 4 for the 12 edges of c."""
        Nx, Ny, Nz = self.Nx, self.Ny, self.Nz
        sigma = np.asarray(sigma, float)
        V = self.hz[:, None, None] * self.hy[None, :, None] * self.hx[None, None, :]
        k, j, i = [a.ravel() for a in np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")]
        c = (k * Ny + j) * Nx + i
        val = 0.25 * (sigma * V).ravel()
        rows, cols, vals = [], [], []
        for dj, dk in ((0, 0), (1, 0), (0, 1), (1, 1)):
            rows.append(self.ex(i, j + dj, k + dk)); cols.append(c); vals.append(val)
        for di, dk in ((0, 0), (1, 0), (0, 1), (1, 1)):
            rows.append(self.ey(i + di, j, k + dk)); cols.append(c); vals.append(val)
        for di, dj in ((0, 0), (1, 0), (0, 1), (1, 1)):
            rows.append(self.ez(i + di, j + dj, k)); cols.append(c); vals.append(val)
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n_edges, Nx * Ny * Nz))

    def loop_source_full(self, i0, i1, j0, j1, k_s, current=1.0):
        """f_e = I l_e s_e on the edges of a counter-clockwise (seen from +z)
        rectangular loop on node lines i0..i1, j0..j1 of node plane k_s."""
        if not (0 < i0 < i1 < self.Nx and 0 < j0 < j1 < self.Ny and 0 < k_s < self.Nz):
            raise ValueError("loop must lie on interior node lines")
        f = np.zeros(self.n_edges)
        i = np.arange(i0, i1)
        f[self.ex(i, j0, k_s)] += current * self.hx[i]
        f[self.ex(i, j1, k_s)] -= current * self.hx[i]
        j = np.arange(j0, j1)
        f[self.ey(i1, j, k_s)] += current * self.hy[j]
        f[self.ey(i0, j, k_s)] -= current * self.hy[j]
        return f

    def receiver_row_full(self, i, j, k_s):
        """Row q with q.u = dB_z/dt on the z-face of cell column (i, j) in plane
        k_s: Faraday's law gives dB_z/dt = -(curl e)_z and the circulation over
        the face divided by its area is (curl e)_z (Sec. 5 observation)."""
        q = np.zeros(self.n_edges)
        A = self.hx[i] * self.hy[j]
        q[self.ex(i, j, k_s)] += self.hx[i]
        q[self.ey(i + 1, j, k_s)] += self.hy[j]
        q[self.ex(i, j + 1, k_s)] -= self.hx[i]
        q[self.ey(i, j, k_s)] -= self.hy[j]
        return -q / A


class Problem:
    """K, M, f and the receiver operator restricted to the interior edges."""

    def __init__(self, wl):
        self.wl = wl
        self.grid = g = YeeGrid(wl.hx, wl.hy, wl.hz)
        self.mask = g.interior()
        self.idx = np.where(self.mask)[0]
        Kf = g.stiffness_full()
        self.K = Kf[self.idx][:, self.idx].tocsr()
        self.sigma = np.asarray(wl.sigma, float)
        self.M = g.mass_full(self.sigma)[self.idx]
        F = [g.loop_source_full(lp.i0, lp.i1, lp.j0, lp.j1, wl.k_s, lp.current) for lp in wl.loops]
        self.F = np.array(F)[:, self.idx].T  # n x n_src
        Q = [g.receiver_row_full(i, j, wl.k_s) for (i, j) in wl.receivers]
        self.Q = sp.csr_matrix(np.array(Q)[:, self.idx]) if Q else sp.csr_matrix((0, len(self.idx)))
        self.n = len(self.idx)

    def mass_derivative(self):
        return self.grid.mass_derivative_full(self.sigma)[self.idx]
