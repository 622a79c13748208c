"""GPU parity of the adjoint gradient (Sec. 4) against the oracle's gradient
and against central finite differences of the GPU forward."""
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


def _misfit_case(n_t=10, m=20):
    wl = W.small_case(7, seed=9, t=W.log_channels(1e-5, 1e-3, n_t))
    wl.receivers = [(2, 2), (3, 3), (4, 2), (2, 4)]
    fit = rkfit.rkfit(wl.t, m)
    s, C = rkfit.shifts_and_coefficients(fit)
    return wl, s, C


def test_adjoint_matches_oracle_gradient(tem):
    wl, s, C = _misfit_case()
    P = yee.Problem(wl)
    rng = np.random.default_rng(0)
    w = rng.standard_normal((len(wl.t), len(wl.receivers)))
    g_or = direct.misfit_gradient(P, s, C, w, method="banded")
    ctx = tem.Context.from_workload(wl)
    ctx.forward(wl.loops, wl.receivers, -s, C, keep_solutions=True)
    g, st = ctx.adjoint(w[None])
    assert st["converged"]
    g = g.ravel()
    err = np.linalg.norm(g - g_or) / np.linalg.norm(g_or)
    print("adjoint rel err %.2e, iterations %d" % (err, st["iterations"]))
    assert err <= 1e-8


def test_adjoint_vs_finite_differences(tem):
    """phi = 1/2 ||d - d_obs||^2; central differences of the GPU forward in
    ln sigma on a few cells (step 1e-3) agree with the adjoint gradient."""
    wl, s, C = _misfit_case(8, 18)
    ctx = tem.Context.from_workload(wl)
    rng = np.random.default_rng(1)
    d0, _ = ctx.forward(wl.loops, wl.receivers, -s, C, keep_solutions=True)
    d_obs = d0 * (1 + 0.2 * rng.standard_normal(d0.shape))
    g, _ = ctx.adjoint(d0 - d_obs)
    h = 1e-3
    cells = [(1, 3, 3), (2, 2, 4), (0, 4, 2), (3, 3, 3)]
    for (k, j, i) in cells:
        vals = []
        for sg in (+1, -1):
            sig = wl.sigma.copy()
            sig[k, j, i] *= np.exp(sg * h)
            ctx.set_conductivity(sig)
            d, _ = ctx.forward(wl.loops, wl.receivers, -s, C)
            vals.append(0.5 * np.sum((d - d_obs) ** 2))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k, j, i]) <= 1e-4 * abs(g[k, j, i]) + 1e-6 * np.abs(g).max(), (k, j, i, fd, g[k, j, i])
    ctx.set_conductivity(wl.sigma)


def test_adjoint_two_sources_sum(tem):
    """The gradient of a two-source misfit is the sum of the per-source ones."""
    wl, s, C = _misfit_case(6, 16)
    wl.loops = [W.Loop(1, 4, 1, 4, 1.0), W.Loop(3, 6, 2, 5, -0.5)]
    ctx = tem.Context.from_workload(wl)
    rng = np.random.default_rng(2)
    w = rng.standard_normal((2, 6, len(wl.receivers)))
    ctx.forward(wl.loops, wl.receivers, -s, C, keep_solutions=True)
    g2, _ = ctx.adjoint(w)
    parts = []
    for q in range(2):
        ctx.forward([wl.loops[q]], wl.receivers, -s, C, keep_solutions=True)
        parts.append(ctx.adjoint(w[q:q + 1])[0])
    assert np.allclose(g2, parts[0] + parts[1], rtol=1e-9, atol=1e-12 * np.abs(g2).max())


def test_adjoint_many_receivers_cocg_path(tem, monkeypatch):
    """The batched COCG path of the adjoint (the library takes it above 86
    receivers; TEM_ADJOINT=cocg selects it here for 70) gives the same
    gradient as the oracle."""
    monkeypatch.setenv("TEM_ADJOINT", "cocg")
    wl = W.small_case(9, seed=9, t=W.log_channels(1e-5, 1e-3, 6))
    wl.receivers = [(i, j) for i in range(9) for j in range(9)][:70]
    fit = rkfit.rkfit(wl.t, 16)
    s, C = rkfit.shifts_and_coefficients(fit)
    P = yee.Problem(wl)
    rng = np.random.default_rng(5)
    w = rng.standard_normal((len(wl.t), len(wl.receivers)))
    g_or = direct.misfit_gradient(P, s, C, w, method="banded")
    ctx = tem.Context.from_workload(wl)
    ctx.forward(wl.loops, wl.receivers, -s, C, keep_solutions=True)
    g, st = ctx.adjoint(w[None])
    err = np.linalg.norm(g.ravel() - g_or) / np.linalg.norm(g_or)
    print("cocg adjoint rel err %.2e" % err)
    assert err <= 1e-8


def test_autograd_function_matches_adjoint(tem):
    """loss.backward() through the autograd Function gives the tem_adjoint
    gradient; a stale context (another forward in between) raises."""
    import torch
    from paper_2506_11657_amd.autograd import receiver_data
    wl, s, C = _misfit_case(6, 16)
    ctx = tem.Context.from_workload(wl)
    rng = np.random.default_rng(5)
    d_obs = torch.from_numpy(rng.standard_normal((1, 6, len(wl.receivers))) * 1e-9)
    m = torch.tensor(np.log(wl.sigma), device="cuda", requires_grad=True)
    d = receiver_data(m, ctx, wl.loops, wl.receivers, -s, C)
    loss = 0.5 * ((d.cpu() - d_obs) ** 2).sum()
    loss.backward()
    d_np, _ = ctx.forward(wl.loops, wl.receivers, -s, C, keep_solutions=True)
    assert np.array_equal(d_np, d.detach().cpu().numpy())
    g_ref, _ = ctx.adjoint(d_np - d_obs.numpy())
    assert np.array_equal(m.grad.cpu().numpy(), g_ref)
    d2 = receiver_data(m, ctx, wl.loops, wl.receivers, -s, C)
    ctx.forward(wl.loops, wl.receivers, -s, C)
    with pytest.raises(RuntimeError):
        d2.sum().backward()


def test_adjoint_recomputes_solutions_when_not_kept(tem):
    """A forward without keep_solutions stores no solutions; the adjoint then
    solves for them again source by source and gives the same gradient, bit
    for bit, as the adjoint of a forward that kept them."""
    wl, s, C = _misfit_case(6, 16)
    wl.loops = [W.Loop(1, 4, 1, 4, 1.0), W.Loop(3, 6, 2, 5, -0.5)]
    ctx = tem.Context.from_workload(wl)
    rng = np.random.default_rng(4)
    w = rng.standard_normal((2, 6, len(wl.receivers)))
    ctx.forward(wl.loops, wl.receivers, -s, C, keep_solutions=True)
    g_keep, _ = ctx.adjoint(w)
    ctx.forward(wl.loops, wl.receivers, -s, C, keep_solutions=False)
    with pytest.raises(tem.TemError):
        ctx.solutions(0)
    g_re, st = ctx.adjoint(w)
    assert np.array_equal(g_keep, g_re)


def test_adjoint_differentiation_config_16(tem):
    """The differentiation workload at 16^3 (blocky current model, 30 surface
    receivers, 40 channels, L2 misfit against the data of a blocky true
    model): the GPU gradient matches the oracle's direct-solve gradient."""
    true_wl, cur_wl = W.cfg_inverse(16)
    fit = rkfit.rkfit(cur_wl.t, cur_wl.degree)
    s, C = rkfit.shifts_and_coefficients(fit)
    ctx = tem.Context.from_workload(true_wl)
    d_obs, _ = ctx.forward(true_wl.loops, true_wl.receivers, -s, C)
    ctx.set_conductivity(cur_wl.sigma)
    d, st = ctx.forward(cur_wl.loops, cur_wl.receivers, -s, C, keep_solutions=True)
    w = d - d_obs
    g, sa = ctx.adjoint(w)
    P = yee.Problem(cur_wl)
    g_or = direct.misfit_gradient(P, s, C, w[0], method="banded")
    err = np.linalg.norm(g.ravel() - g_or) / np.linalg.norm(g_or)
    print("16^3 differentiation workload: %d receivers, adjoint rel err %.2e, %d + %d seed iterations"
          % (len(cur_wl.receivers), err, st["iterations"], sa["iterations"]))
    assert len(cur_wl.receivers) == 30 and err <= 1e-8
