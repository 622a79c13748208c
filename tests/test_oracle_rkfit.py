"""Pins of the oracle's shared-pole family against the numbers the paper
prints (Table 1, the solve counts of Sec. 3 and 5, the pole pair of Fig. 1)
and against properties fixed by the mathematics."""
import json
import os

import numpy as np
import pytest

from oracle import rkfit as R

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TABLE = json.load(open(os.path.join(GOLD, "table1.json")))
COUNTS = json.load(open(os.path.join(GOLD, "paper_counts.json")))
SLOW = os.environ.get("TEM_SLOW") == "1"


def test_table1_first_column_from_halphen():
    """Table 1, ratio 1: the [m/m] degrees 2, 4, 7, 9, 11 follow from the
    asymptotic best-approximation error 2 H^(-m-1/2) (Sec. 3.3)."""
    got = [R.single_time_degree(tol) for tol in TABLE["tolerances"]]
    assert got == TABLE["degree"]["1"]


def test_table1_break_even_averages():
    """Table 1 bottom row: avg over tolerances of ceil(m_hat/2)/ceil(m/2)."""
    m = TABLE["degree"]["1"]
    for key, ref in TABLE["avg_K_star"].items():
        ks = [R.break_even(mh, mm) for mh, mm in zip(TABLE["degree"][key], m)]
        assert round(float(np.mean(ks)), 1) == ref


def test_paper_solve_counts():
    c = COUNTS
    assert R.solve_counts(7, 31, 27) == (c["single_time_m7_K31_solves"], c["rkfit_ratio1e3_tol1e-6_solves"])
    single, shared = R.solve_counts(14, 31, 38)
    assert single == c["single_time_m14_K31_solves"] and shared == c["rkfit_m38_solves"]
    assert single / shared > c["solve_ratio_lower_bound"]


def _table_cases():
    cases = []
    for key in ["1e1", "1e2", "1e3", "1e4", "1e5"]:
        for tol, m in zip(TABLE["tolerances"], TABLE["degree"][key]):
            cases.append((float(key), tol, m))
    return cases


FAST_CASES = [(1e3, 1e-6, 27), (1e3, 1e-8, 35), (1e4, 1e-8, 44), (1e1, 1e-6, 14)]


@pytest.mark.parametrize("ratio,tol,m", _table_cases() if SLOW else FAST_CASES)
def test_table1_degree_reaches_tolerance(ratio, tol, m):
    """Table 1: the shared-pole family of the listed degree reaches the listed
    uniform error on 31 log-spaced channels.  The surrogate and start poles of
    the paper's runs are not stated; 23 of the 25 entries are met exactly and
    the remaining two (ratio 10, degrees 9 and 18) within 14 %, so the bound
    allows a factor 1.2."""
    tau = np.logspace(-np.log10(ratio), 0, TABLE["channels_per_fit"])
    fit = R.rkfit(tau, m)
    assert fit["err"].max() <= 1.2 * tol


def test_fig1_poles_pairs_and_printed_pair():
    """Fig. 1 (bottom): degree 28 on [1e-3, 1] with 31 channels gives 14
    conjugate pairs away from x >= 0, and the printed pair -7.574 +- 12.45i is
    among them (within 10 %).  The caption calls it the pair closest to the
    origin; this reading of the unstated surrogate and start poles does not
    reproduce that: its closest pair lies near the negative real axis
    (|Im| < 3, |xi| about 10).  Thirty variants (surrogate range and sample
    count, start poles on a 60 degree ray or at infinity, 10 or 20 sweeps,
    best or last sweep, reflection into Re xi < 0) all gave such a near-real
    closest pair, so the difference is kept as a stated deviation and pinned
    here as measured."""
    c = COUNTS
    t = np.logspace(np.log10(c["fig1_window"][0]), np.log10(c["fig1_window"][1]), c["fig1_channels"])
    fit = R.rkfit(t, c["fig1_degree"])
    xi = fit["xi"]
    assert fit["pairs"].sum() == c["fig1_pair_count"] and len(xi) == c["fig1_pair_count"]
    target = complex(*c["fig1_closest_pair"])
    assert np.min(np.abs(xi - target)) / abs(target) < 0.10
    closest = xi[np.argmin(np.abs(xi))]
    assert abs(closest) < abs(target) and abs(closest.imag) < 3.0
    # distance from the spectral region [0, inf)
    dist = np.where(xi.real >= 0, np.abs(xi.imag), np.abs(xi))
    assert np.all(dist > 1.0)


def test_time_scaling_invariance():
    """exp(-t x) = exp(-(t/s)(s x)): fitting s*t gives poles xi/s, residues
    alpha/s and the same errors (s a power of two, so t/t_max is unchanged)."""
    t = np.logspace(-5, -2, 12)
    s = 1024.0
    a = R.rkfit(t, 20)
    b = R.rkfit(t * s, 20)
    assert np.allclose(b["xi"], a["xi"] / s, rtol=1e-13)
    assert np.allclose(b["alpha"], a["alpha"] / s, rtol=1e-12)
    assert np.array_equal(a["err"], b["err"])


@pytest.mark.parametrize("m", [4, 7, 10])
def test_single_time_near_best(m):
    """One channel: the subdiagonal fit is within a small factor of the best
    [m/m] approximation error 2 H^(-m-1/2) (Sec. 3.3)."""
    fit = R.rkfit(np.array([1.0]), m)
    assert fit["err"][0] <= 3.0 * 2.0 * R.HALPHEN ** (-m - 0.5)


def test_error_measure_matches_brute_force():
    """eq. (error) on random x >= 0 never exceeds the reported per-channel
    error by more than the resolution of the dense check set."""
    t = np.logspace(-3, 0, 10)
    fit = R.rkfit(t, 20)
    rng = np.random.default_rng(0)
    x = 10 ** rng.uniform(-6, 11, 20000)
    tau = t / t.max()
    xi, alpha = fit["xi"] * t.max(), fit["alpha"] * t.max()
    direct = np.zeros((len(x), len(t)))
    for p, a, pair in zip(xi, alpha, fit["pairs"]):
        term = a[None, :] / (x[:, None] - p)
        direct += 2 * term.real if pair else term.real
    e = np.abs(np.exp(-np.outer(x, tau)) - direct).max(axis=0)
    assert np.all(e <= 1.05 * fit["err"])


def test_conjugate_symmetry_of_full_family():
    """Writing out both poles of each pair with conjugate residues gives a real
    rational function; the real-arithmetic least squares guarantees it."""
    t = np.logspace(-4, 0, 8)
    fit = R.rkfit(t, 16)
    x = np.linspace(0, 50, 101)
    full = np.zeros((len(x), len(t)), complex)
    for p, a, pair in zip(fit["xi"], fit["alpha"], fit["pairs"]):
        full += a[None, :] / (x[:, None] - p)
        if pair:
            full += a.conj()[None, :] / (x[:, None] - np.conj(p))
    assert np.abs(full.imag).max() <= 1e-12 * np.abs(full.real).max()


def test_weighted_rkfit_moves_accuracy_to_late_channels():
    """Sec. 5.2: weights w_j ~ t_j^{5/2} in eq. (rkfit) offset the t^{-5/2}
    late-time decay of dB_z/dt.  At degree 38 on [1e-5, 1e-2] (20 channels),
    the weighted fit lowers the error of eq. (error) at the last channel by
    more than 100x and raises it at the first (measured: 9.4e-10 -> 4.2e-12 and
    1.3e-9 -> 1.1e-7), it beats the unweighted fit on the weighted uniform error
    of eq. (uniform_error) that it targets, and the relative error bound
    err_k / t_k^{-5/2} of a transient decaying like t^{-5/2} is flatter (its
    worst channel is lower).  The host fit (tem_poles with w) agrees with the
    oracle's to a factor of 5 on every channel."""
    from paper_2506_11657_amd import tem as T
    t = np.logspace(-5, -2, 20)
    w = (t / t.max()) ** 2.5
    plain = R.rkfit(t, 38)
    weighted = R.rkfit(t, 38, w=w)
    e0, e1 = plain["err"], weighted["err"]
    assert e1[-1] <= 1e-2 * e0[-1] and e1[0] >= e0[0]
    assert (w * e1).max() <= (w * e0).max()
    decay = (t / t[0]) ** -2.5
    assert (e1 / decay).max() < (e0 / decay).max()
    _, _, eh = T.poles(t, 38, w=w)
    assert np.all(eh <= 5 * e1) and np.all(e1 <= 5 * eh)
