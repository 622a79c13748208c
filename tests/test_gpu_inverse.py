"""GPU Jacobian action (tem_jacobian_apply) against the oracle's, the adjoint
identity on the GPU, and a Gauss-Newton step with CGLS and Tikhonov rows on
the 16^3 differentiation workload (Sec. 4)."""
import numpy as np
import pytest

import tem_workloads as W
from oracle import direct, rkfit, yee

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_11657_amd import tem as T
    T.lib()
    return T


def _case():
    wl = W.small_case(7, seed=12, t=W.log_channels(1e-5, 1e-3, 10))
    wl.receivers = [(2, 2), (3, 3), (4, 2)]
    fit = rkfit.rkfit(wl.t, 18)
    s, C = rkfit.shifts_and_coefficients(fit)
    return wl, s, C


def test_jacobian_apply_matches_oracle(tem):
    """J dm on the GPU (sensitivity systems by batched FP64 COCG) against the
    oracle's direct solves, per channel and receiver with the bar of the
    forward data: 1e-8 |J dm| + 1e-9 ||q||_{M^-1} S'_k, S'_k = sum_j |c_jk| ||dx_j||_M
    (the size of the residue-sum terms of the sensitivity)."""
    wl, s, C = _case()
    P = yee.Problem(wl)
    ctx = tem.Context.from_workload(wl)
    ctx.forward(wl.loops, wl.receivers, -s, C, keep_solutions=True)
    rng = np.random.default_rng(3)
    dm = np.zeros(wl.sigma.shape)
    n_earth = wl.k_s
    dm[:n_earth] = rng.standard_normal((n_earth,) + wl.sigma.shape[1:])
    jg, st = ctx.jacobian_apply(dm)
    X = direct.solve_shifted(P, s, P.F[:, 0], "banded")
    jo = direct.jacobian_apply(P, s, C, dm.ravel(), X=X, method="banded")
    dM = P.mass_derivative() @ dm.ravel()
    dX = np.stack([-direct.solve_shifted(P, [sj], sj * dM * X[:, j], "banded")[:, 0] for j, sj in enumerate(s)], 1)
    Sk = np.abs(C).T @ direct.m_norm(P, dX)
    qn = np.sqrt(np.asarray(P.Q.multiply(P.Q) @ (1.0 / P.M)).ravel())
    err = np.abs(jg[0] - jo)
    print("J dm: COCG iterations %d, max |err| / |J dm| %.2e, max err / floor %.2e"
          % (st["iterations"], (err / np.abs(jo)).max(), (err / np.outer(Sk, qn)).max()))
    assert np.all(err <= 1e-8 * np.abs(jo) + 1e-9 * np.outer(Sk, qn))
    # <w, J dm> = <J^T w, dm>, both on the GPU
    w = rng.standard_normal(jg.shape)
    g, _ = ctx.adjoint(w)
    lhs, rhs = float(np.sum(w * jg)), float(np.sum(g * dm))
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs)


def test_jacobian_apply_needs_kept_solutions(tem):
    wl, s, C = _case()
    ctx = tem.Context.from_workload(wl)
    ctx.forward(wl.loops, wl.receivers, -s, C)
    with pytest.raises(tem.TemError) as e:
        ctx.jacobian_apply(np.zeros(wl.sigma.shape))
    assert e.value.status == tem.TEM_ESTATE


def test_gauss_newton_cgls_step_reduces_misfit(tem):
    """One Gauss-Newton step on the 16^3 differentiation workload (blocky true
    and current earth models, 30 surface receivers, 40 channels): CGLS with 3
    iterations on the earth cells, data weighted by 1/|d_obs| (the channels
    span orders of magnitude), Tikhonov rows towards the current model; the
    accepted step lowers the regularized misfit by at least 20%."""
    from paper_2506_11657_amd.inversion import gauss_newton_step
    true_wl, cur_wl = W.cfg_inverse(16)
    xi, c, err = tem.poles(cur_wl.t, cur_wl.degree)
    ctx = tem.Context.from_workload(true_wl)
    d_obs, _ = ctx.forward(true_wl.loops, true_wl.receivers, xi, c)
    wd = 1.0 / (np.abs(d_obs) + 1e-6 * np.abs(d_obs).max())
    active = np.zeros(cur_wl.sigma.shape, bool)
    active[:cur_wl.k_s] = True
    sig1, info = gauss_newton_step(ctx, cur_wl, xi, c, d_obs, active, lam=1e-2, wd=wd, cgls_iters=3)
    print("Gauss-Newton: misfit %.4e -> %.4e at step %.3f; CGLS normal residuals %s"
          % (info["phi0"], info["phi"], info["step"], " ".join("%.2e" % v for v in info["cgls_normal_residuals"])))
    assert info["step"] > 0 and info["phi"] <= 0.8 * info["phi0"]
    m_true, m0, m1 = (np.log(x)[active] for x in (true_wl.sigma, cur_wl.sigma, sig1))
    print("model error ||m - m_true||: %.3f -> %.3f" % (np.linalg.norm(m0 - m_true), np.linalg.norm(m1 - m_true)))
