"""The 64^3 graded workload at its full size, in the configuration the
benchmark times: FP64, 64-iteration blocks, default rtol, MFMA contraction into
full fields, the centre receiver.

A direct solve of one 64^3 shifted system does not fit in memory (band ~24k),
so parity here rests on properties that hold at any size, evaluated with the
oracle's own assembled operators (CSR K, lumped M, loop source, receiver row):

  * residual: rho_j = ||f - (K + s_j M) x_j||_{M^-1} / ||f||_{M^-1} of each
    returned solution equals the true residual the library reports (both are
    the scaled residual of Sec. 3.2's shifted system, computed in different
    rounding orders) and is small.  Since A = M^-1/2 K M^-1/2 is symmetric
    PSD, ||(A + s)^-1|| <= 1/dist(-s, [0, inf)), which turns rho_j into a
    rigorous bound on ||x_j - x*_j||_M; it is printed per channel;
  * contraction: every stored field value equals Re sum_j c_jk x_j of the
    returned solutions (1e-13 of the term sizes), and edges outside the
    interior are exactly zero;
  * receivers: the data equal the oracle's receiver row applied to the fields
    (1e-11 relative, 1e-13 of the residue terms at the receiver);
  * physics: ||u(t_k)||_M does not increase with k beyond the approximation
    error of the fit (e^{-tA} is a contraction for A PSD, Sec. 2.2), and the
    step-off response dB_z/dt at the loop centre is negative on every channel
    resolved well above that error.
"""
import numpy as np
import pytest

import tem_workloads as W
from oracle import direct, rkfit, yee

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def run():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_11657_amd import tem
    tem.lib()
    wl = W.cfg_graded64()
    fit = rkfit.rkfit(wl.t, wl.degree)
    s, C = rkfit.shifts_and_coefficients(fit)
    P = yee.Problem(wl)
    ctx = tem.Context.from_workload(wl)
    T = len(wl.t)
    fields = torch.zeros((1, T, ctx.n_storage), dtype=torch.float64, device="cuda")
    print("graded64: n = %d unknowns, J = %d shifts, T = %d channels" % (P.n, len(s), T), flush=True)
    data, st = ctx.forward(wl.loops, wl.receivers, -s, C, fields=fields, block=64, keep_solutions=True)
    print("seed iterations %d, max true residual %.2e" % (st["iterations"], max(st["true_res"])), flush=True)
    X = ctx.solutions(0)
    U = fields[0].cpu().numpy()
    del fields
    return wl, fit, s, C, P, data, st, X, U


def test_graded64_residuals_in_oracle_operators(run):
    wl, fit, s, C, P, data, st, X, U = run
    assert st["converged"]
    f = P.F[:, 0]
    fn = np.sqrt(np.sum(f * f / P.M))
    absK = abs(P.K)
    rho = np.empty(len(s))
    floor = np.empty(len(s))
    for j in range(len(s)):
        x = X[j, P.idx]
        r = f - (P.K @ x + s[j] * (P.M * x))
        rho[j] = np.sqrt(np.sum(np.abs(r) ** 2 / P.M)) / fn
        # rounding floor of evaluating r in FP64: eps times the sizes of its terms
        terms = absK @ np.abs(x) + abs(s[j]) * P.M * np.abs(x) + np.abs(f)
        floor[j] = 2.2e-16 * 16 * np.sqrt(np.sum(terms ** 2 / P.M)) / fn
    gpu = np.asarray(st["true_res"])
    print("rho (oracle operators):", " ".join("%.2e" % v for v in rho))
    print("rounding floor:        ", " ".join("%.1e" % v for v in floor))
    assert np.all(np.abs(rho - gpu) <= 1e-3 * gpu + floor)
    assert rho.max() <= 1e-7
    # ||x_j - x*_j||_M <= rho_j ||f||_{M^-1} / dist(-s_j, [0, inf))
    dist = np.where(s.real >= 0, np.abs(s), np.abs(s.imag))
    ebound = rho * fn / dist
    xn = direct.m_norm(P, X[:, P.idx].T)
    un = direct.m_norm(P, U[:, P.idx].T)
    Sk = np.abs(C).T @ xn
    Ek = np.abs(C).T @ ebound
    print("per-shift error bound / ||x_j||_M:", " ".join("%.1e" % v for v in ebound / xn))
    print("channel error bound / ||u_k||_M:", " ".join("%.1e" % v for v in Ek / un))
    print("S_k / ||u_k||_M:", " ".join("%.1e" % v for v in Sk / un))


def test_graded64_fields_are_the_residue_sum(run):
    wl, fit, s, C, P, data, st, X, U = run
    assert np.all(U[:, ~P.mask] == 0.0)
    Xi = X[:, P.idx].T
    ref = direct.contract(Xi, C).T                  # (T, n)
    scale = (np.abs(Xi) @ np.abs(C)).T
    err = np.abs(U[:, P.idx] - ref)
    worst = np.unravel_index(np.argmax(err / (scale + 1e-300)), err.shape)
    print("max |U - Re XC| / term size %.2e at channel %d" % ((err / (scale + 1e-300))[worst], worst[0]))
    assert np.all(err <= 1e-13 * scale)


def test_graded64_receiver_and_decay(run):
    wl, fit, s, C, P, data, st, X, U = run
    Ui = U[:, P.idx]                                # (T, n)
    d = P.Q @ Ui.T                                  # (n_rx, T)
    xn = direct.m_norm(P, X[:, P.idx].T)
    Sk = np.abs(C).T @ xn
    qn = np.sqrt(np.asarray(P.Q.multiply(P.Q) @ (1.0 / P.M)).ravel())
    # the library sums the residue terms at the receiver, the oracle sums the
    # fields: late channels cancel, so the floor is the size of those terms
    Xi = X[:, P.idx].T
    scale = ((np.abs(P.Q) @ np.abs(Xi)) @ np.abs(C))     # (n_rx, T)
    assert np.all(np.abs(data[0].T - d) <= 1e-11 * np.abs(d) + 1e-13 * scale)
    un = direct.m_norm(P, Ui.T)
    bn = direct.m_norm(P, P.F[:, 0] / P.M)
    err = fit["err"]
    # the fit's uniform error plus the FP64 parity bar per channel
    dev = err * bn + 1e-8 * un + 1e-10 * Sk
    print("||u_k||_M:", " ".join("%.2e" % v for v in un))
    print("dB_z/dt at the centre:", " ".join("%.2e" % v for v in data[0, :, 0]))
    assert np.all(np.diff(un) <= dev[:-1] + dev[1:])
    resolved = un > 1e3 * (err * bn + 1e-10 * Sk)
    dv = data[0, :, 0]
    dres = np.abs(dv) > 1e3 * (err * bn + 1e-10 * Sk) * qn[0]
    print("resolved channels: %d by norm, %d at the receiver" % (resolved.sum(), dres.sum()))
    assert resolved.sum() >= 10 and dres.sum() >= 10
    assert np.all(dv[dres] < 0)
