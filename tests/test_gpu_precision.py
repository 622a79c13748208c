"""GPU parity of precision 1 (FP64 iterates with complex FP32 search
directions in the multi-shift sweep, FP64 true residuals, FP64 residual
refinement with FP32 batched COCG corrections; contraction and receivers in
FP64) against the CPU oracle.

Bar (FP32 form): per-shift ||x_j - x_or,j||_M <= 1e-6 ||x_or,j||_M and per channel
    ||u_gpu(t_k) - u_or(t_k)||_M <= 1e-5 ||u_or(t_k)||_M + 1e-6 S_k,
with S_k = sum_j |c_jk| ||x_j||_M the size of the residue-sum terms.  The
M-norm error of a shift is set by the FP32 rounding of its search direction
(a few 1e-8 relative, measured in a NumPy model of the sweep on the 1e-8 S/m
ragged grid), well inside the bar; a channel whose terms are at most 10x its
value (S_k <= 10 ||u_k||) therefore meets 2e-5 relative outright, later
channels cancel (S_k / ||u_k|| reaches 1e10 at 16^3) and are checked against
the eta S_k floor.  Refinement drives the FP64 residual to the default 1e-5
(the rounding noise of the stiff air modes dominates it; FP32 corrections stop
improving it near 1e-6 on grids with 1e-8 S/m air).
"""
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


def _fit(t, m):
    f = rkfit.rkfit(t, m)
    s, C = rkfit.shifts_and_coefficients(f)
    return -s, s, C


def _channel_errors(P, X, Xo, C):
    xn = direct.m_norm(P, Xo)
    U, Uo = direct.contract(X, C), direct.contract(Xo, C)
    eu = direct.m_norm(P, U - Uo)
    un = direct.m_norm(P, Uo)
    Sk = np.abs(C).T @ xn
    return eu, un, Sk, direct.m_norm(P, X - Xo) / xn


def test_precision1_parity_plain16(tem):
    wl = W.cfg_plain16()
    xi, s, C = _fit(wl.t, wl.degree)
    P = yee.Problem(wl)
    ctx = tem.Context.from_workload(wl)
    data, st = ctx.forward(wl.loops, wl.receivers, xi, C, precision=1, keep_solutions=True)
    X = ctx.solutions(0)[:, P.idx].T
    Xo = direct.solve_shifted(P, s, P.F[:, 0], "banded")
    eu, un, Sk, ex = _channel_errors(P, X, Xo, C)
    rel = eu / un
    print("precision 1: sweep iterations %d, refinement passes %d, max true res %.2e, max shift err %.2e"
          % (st["iterations"], st["refine_passes"], max(st["true_res"]), ex.max()))
    print("per-channel relative error vs oracle:", " ".join("%.1e" % v for v in rel))
    assert st["converged"] and max(st["true_res"]) <= 1e-5
    assert ex.max() <= 1e-6
    assert np.all(eu <= 1e-5 * un + 1e-6 * Sk)
    resolved = Sk <= 10 * un
    assert resolved.sum() >= 3 and np.all(rel[resolved] <= 2e-5)


def test_precision1_matches_fp64_ragged(tem):
    """Multi-tile ragged grid (air 1e-5 S/m), two sources: precision 1 against
    the FP64 GPU path (itself oracle-checked) channel by channel, and receivers."""
    wl = W.ragged29(1e-5)
    xi, s, C = _fit(wl.t, 16)
    P = yee.Problem(wl)
    ctx = tem.Context.from_workload(wl)
    d64, _ = ctx.forward(wl.loops, wl.receivers, xi, C, keep_solutions=True)
    X64 = [ctx.solutions(q)[:, P.idx].T for q in range(2)]
    d32, st = ctx.forward(wl.loops, wl.receivers, xi, C, precision=1, keep_solutions=True)
    assert st["converged"] and max(st["true_res"]) <= 1e-5
    qn = np.sqrt(np.asarray(P.Q.multiply(P.Q) @ (1.0 / P.M)).ravel())
    for q in range(2):
        X32 = ctx.solutions(q)[:, P.idx].T
        eu, un, Sk, ex = _channel_errors(P, X32, X64[q], C)
        print("source %d: max shift err %.2e, channel errs %s" % (q, ex.max(), " ".join("%.1e" % v for v in eu / un)))
        assert ex.max() <= 1e-6
        assert np.all(eu <= 1e-5 * un + 1e-6 * Sk)
        assert np.all(np.abs(d32[q] - d64[q]) <= 1e-5 * np.abs(d64[q]) + 1e-6 * np.outer(Sk, qn))


def test_precision1_stiff_grid_parity_vs_oracle(tem):
    """The ragged multi-tile grid with the paper's 1e-8 S/m air (about 1.6e4
    seed iterations, air modes 1e10 above the earth's), two sources: the call
    converges to the default FP64 residual target, every shift and channel of
    both sources is within the FP32-form bar of the oracle's direct solves, the
    receivers too, and further refinement passes never leave a shift worse."""
    wl = W.ragged29()
    xi, s, C = _fit(wl.t, 16)
    P = yee.Problem(wl)
    ctx = tem.Context.from_workload(wl)
    _, st1 = ctx.forward(wl.loops, wl.receivers, xi, C, precision=1, refine_max=1, allow_noconv=True)
    data, st = ctx.forward(wl.loops, wl.receivers, xi, C, precision=1, keep_solutions=True)
    print("sweep %d iterations; FP64 residual after one pass %.2e, after refinement %.2e (%d passes, %s)"
          % (st["iterations"], max(st1["true_res"]), max(st["true_res"]), st["refine_passes"], st["status"]))
    assert st["converged"] and max(st["true_res"]) <= 1e-5
    assert np.all(np.array(st["true_res"]) <= np.array(st1["true_res"]) * (1 + 1e-6))
    qn = np.sqrt(np.asarray(P.Q.multiply(P.Q) @ (1.0 / P.M)).ravel())
    for q in range(2):
        X = ctx.solutions(q)[:, P.idx].T
        Xo = direct.solve_shifted(P, s, P.F[:, q], "splu")
        eu, un, Sk, ex = _channel_errors(P, X, Xo, C)
        d_or = (P.Q @ direct.contract(Xo, C)).T
        print("source %d: max shift M-norm err %.2e, channel errs %s" % (q, ex.max(), " ".join("%.1e" % v for v in eu / un)))
        assert ex.max() <= 1e-6
        assert np.all(eu <= 1e-5 * un + 1e-6 * Sk)
        assert np.all(np.abs(data[q] - d_or) <= 1e-5 * np.abs(d_or) + 1e-6 * np.outer(Sk, qn))
        resolved = Sk <= 10 * un
        assert resolved.sum() >= 3 and np.all(eu[resolved] <= 2e-5 * un[resolved])


def test_precision1_refinement_reaches_requested_rtol(tem):
    """The default target (1e-5) is met; a tighter one runs at least as many
    passes, never leaves a shift worse, and either meets it (converged) or
    says so (TEM_ENOCONV) with the floor it reached printed; 1e-8 asks for the
    FP64 path's own attainable level; an unreachable target with one pass is
    reported."""
    wl = W.small_case(9, seed=3, t=W.log_channels(1e-5, 1e-3, 10))
    xi, s, C = _fit(wl.t, 16)
    ctx = tem.Context.from_workload(wl)
    _, st5 = ctx.forward(wl.loops, wl.receivers, xi, C, precision=1)
    assert st5["converged"] and max(st5["true_res"]) <= 1e-5
    for rtol in (1e-7, 1e-8):
        _, stt = ctx.forward(wl.loops, wl.receivers, xi, C, precision=1, rtol=rtol, allow_noconv=True)
        print("rtol %.0e: %d passes (default target: %d), max FP64 residual %.2e, %s"
              % (rtol, stt["refine_passes"], st5["refine_passes"], max(stt["true_res"]), stt["status"]))
        assert stt["refine_passes"] >= st5["refine_passes"]
        assert np.all(np.array(stt["true_res"]) <= np.array(st5["true_res"]) * (1 + 1e-6))
        if stt["converged"]:
            assert max(stt["true_res"]) <= rtol
        else:
            assert stt["status"] == "TEM_ENOCONV" and max(stt["true_res"]) > rtol
    _, st1 = ctx.forward(wl.loops, wl.receivers, xi, C, precision=1, rtol=1e-13, refine_max=1, allow_noconv=True)
    assert st1["refine_passes"] == 1
    assert st1["status"] == "TEM_ENOCONV" and not st1["converged"]
