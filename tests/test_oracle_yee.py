"""Pins of the oracle's Yee-grid operators against facts fixed by the
mathematics (curl grad = 0, the Yee cavity spectrum, Stokes' theorem,
axis-permutation symmetry), not against the oracle's own formulas."""
import itertools

import numpy as np
import pytest

import tem_workloads as W
from oracle import yee


def _grid(hx, hy, hz):
    return yee.YeeGrid(np.asarray(hx, float), np.asarray(hy, float), np.asarray(hz, float))


def test_curl_of_gradient_vanishes():
    rng = np.random.default_rng(0)
    g = _grid(rng.uniform(1, 3, 4), rng.uniform(1, 3, 5), rng.uniform(1, 3, 3))
    C, w = g.curl()
    G = g.gradient()
    CG = (C @ G).toarray()
    assert np.abs(CG).max() <= 1e-13 * np.abs(C).max() * np.abs(G).max()
    assert np.all(w > 0)


def test_stiffness_symmetric_psd_and_null_space():
    rng = np.random.default_rng(1)
    g = _grid(rng.uniform(1, 3, 3), rng.uniform(1, 3, 4), rng.uniform(1, 3, 3))
    m = g.interior()
    K = g.stiffness_full()[m][:, m].toarray()
    assert np.allclose(K, K.T, rtol=0, atol=1e-14 * np.abs(K).max())
    lam = np.linalg.eigvalsh(K)
    assert lam.min() > -1e-12 * lam.max()
    # null space = gradients of interior-node potentials
    n_int_nodes = (g.Nx - 1) * (g.Ny - 1) * (g.Nz - 1)
    assert np.sum(lam < 1e-10 * lam.max()) == n_int_nodes


@pytest.mark.parametrize("N", [(3, 4, 5), (4, 4, 4)])
def test_yee_cavity_spectrum(N):
    """Uniform cells and conductivity in a PEC box: the nonzero eigenvalues of
    M^-1 K are (4/(mu0 sigma)) sum_a sin^2(p_a pi / 2N_a)/h_a^2, with
    multiplicity 2 when all three indices are nonzero and 1 when exactly one
    is zero (discrete TE/TM cavity modes)."""
    Nx, Ny, Nz = N
    h = (10.0, 12.0, 15.0)
    sigma = 0.05
    g = _grid([h[0]] * Nx, [h[1]] * Ny, [h[2]] * Nz)
    m = g.interior()
    K = g.stiffness_full()[m][:, m].toarray()
    M = g.mass_full(np.full((Nz, Ny, Nx), sigma))[m]
    lam = np.sort(np.linalg.eigvalsh(K / np.sqrt(M)[:, None] / np.sqrt(M)[None, :]))
    ref = []
    for p, q, r in itertools.product(range(Nx), range(Ny), range(Nz)):
        zeros = (p == 0) + (q == 0) + (r == 0)
        mult = {0: 2, 1: 1}.get(zeros, 0)
        val = 4.0 / (yee.MU0 * sigma) * (np.sin(p * np.pi / (2 * Nx)) ** 2 / h[0] ** 2
                                         + np.sin(q * np.pi / (2 * Ny)) ** 2 / h[1] ** 2
                                         + np.sin(r * np.pi / (2 * Nz)) ** 2 / h[2] ** 2)
        ref += [val] * mult
    ref = np.sort(ref)
    nz = lam[lam > 1e-9 * lam.max()]
    assert len(nz) == len(ref)
    assert np.allclose(nz, ref, rtol=1e-10)


def _linear_field(g, B0=1.0):
    """Edge-midpoint samples of e = B0 (-y/2, x/2, 0): curl e = B0 z-hat."""
    x = np.concatenate([[0.0], np.cumsum(g.hx)])
    y = np.concatenate([[0.0], np.cumsum(g.hy)])
    ex = np.broadcast_to(-B0 * y[None, :, None] / 2, (g.Nz + 1, g.Ny + 1, g.Nx)).ravel()
    ey = np.broadcast_to(B0 * x[None, None, :] / 2, (g.Nz + 1, g.Ny, g.Nx + 1)).ravel()
    ez = np.zeros(g.n_ez)
    return np.concatenate([ex, ey, ez])


def test_receiver_row_is_minus_curl_z():
    """Stokes: the circulation of a field with constant curl B0 over any face
    equals B0 times its area, so q.u = dB_z/dt = -(curl e)_z = -B0."""
    rng = np.random.default_rng(2)
    g = _grid(rng.uniform(5, 20, 6), rng.uniform(5, 20, 7), rng.uniform(5, 20, 5))
    u = _linear_field(g, 3.0)
    for (i, j) in [(0, 0), (2, 3), (5, 6)]:
        assert np.isclose(g.receiver_row_full(i, j, 2) @ u, -3.0, rtol=1e-13)


def test_loop_source_orientation_and_area():
    """f.e = I * (circulation of e around the loop) = I * B0 * loop area for
    e with constant curl B0 z-hat (counter-clockwise seen from +z), and a
    closed loop carries no charge: G^T f = 0."""
    rng = np.random.default_rng(3)
    g = _grid(rng.uniform(5, 20, 8), rng.uniform(5, 20, 9), rng.uniform(5, 20, 6))
    f = g.loop_source_full(2, 6, 3, 7, 3, current=2.0)
    area = g.hx[2:6].sum() * g.hy[3:7].sum()
    assert np.isclose(f @ _linear_field(g, 1.0), 2.0 * area, rtol=1e-13)
    assert np.abs(g.gradient().T @ f).max() < 1e-14 * np.abs(f).max()


def _components(g, v):
    ex = v[:g.n_ex].reshape(g.Nz + 1, g.Ny + 1, g.Nx)
    ey = v[g.n_ex:g.n_ex + g.n_ey].reshape(g.Nz + 1, g.Ny, g.Nx + 1)
    ez = v[g.n_ex + g.n_ey:].reshape(g.Nz, g.Ny + 1, g.Nx + 1)
    return ex, ey, ez


def test_mass_axis_swap_and_reflection_equivariance():
    """Swapping x and y (sigma transposed, widths swapped) must swap the Ex and
    Ey mass entries; reflecting x must reflect them.  A cell chosen from the
    wrong side or axis for an edge breaks one of these."""
    rng = np.random.default_rng(4)
    hx, hy, hz = rng.uniform(5, 20, 4), rng.uniform(5, 20, 5), rng.uniform(5, 20, 3)
    sigma = 10 ** rng.uniform(-3, 0, (3, 5, 4))
    g = _grid(hx, hy, hz)
    mx, my, mz = _components(g, g.mass_full(sigma))
    gs = _grid(hy, hx, hz)
    sx, sy, sz = _components(gs, gs.mass_full(np.transpose(sigma, (0, 2, 1))))
    assert np.allclose(sx, np.transpose(my, (0, 2, 1)), rtol=1e-14)
    assert np.allclose(sy, np.transpose(mx, (0, 2, 1)), rtol=1e-14)
    assert np.allclose(sz, np.transpose(mz, (0, 2, 1)), rtol=1e-14)
    gr = _grid(hx[::-1], hy, hz)
    rx, ry, rz = _components(gr, gr.mass_full(sigma[:, :, ::-1]))
    assert np.allclose(rx, mx[:, :, ::-1], rtol=1e-14)
    assert np.allclose(ry, my[:, :, ::-1], rtol=1e-14)
    # uniform field e_x: the lumped energy equals the exact integral of sigma
    assert np.isclose(mx.sum(), (sigma * hz[:, None, None] * hy[None, :, None] * hx[None, None, :]).sum(), rtol=1e-13)


def test_stiffness_axis_swap_equivariance():
    rng = np.random.default_rng(5)
    hx, hy, hz = rng.uniform(5, 20, 3), rng.uniform(5, 20, 4), rng.uniform(5, 20, 3)
    g, gs = _grid(hx, hy, hz), _grid(hy, hx, hz)
    u = rng.standard_normal(g.n_edges)
    ux, uy, uz = _components(g, u)
    us = np.concatenate([np.transpose(uy, (0, 2, 1)).ravel(), np.transpose(ux, (0, 2, 1)).ravel(),
                         np.transpose(uz, (0, 2, 1)).ravel()])
    # a swap of x and y is a reflection: it flips the orientation of circulations,
    # which the quadratic form does not see
    e1 = u @ (g.stiffness_full() @ u)
    e2 = us @ (gs.stiffness_full() @ us)
    assert np.isclose(e1, e2, rtol=1e-12)


def test_problem_restriction_matches_storage():
    wl = W.small_case(5)
    P = yee.Problem(wl)
    assert P.n == 3 * 5 * 4 * 4
    assert P.F.shape == (P.n, 1)
    assert P.Q.shape == (1, P.n)
    # interior loop: source charge-free on the interior-node gradient
    G = P.grid.gradient()[P.idx]
    assert np.abs(G.T @ P.F[:, 0]).max() < 1e-14 * np.abs(P.F).max()
