"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, validates arguments without touching a GPU, and its host
RKFIT (tem_poles) meets the same paper pins as the oracle."""
import json
import os
import re

import numpy as np
import pytest

from paper_2506_11657_amd import tem as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


def _declared():
    src = open(os.path.join(ROOT, "include", "tem.h")).read()
    return sorted(set(re.findall(r"\b(tem_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    L = T.lib()
    names = _declared()
    assert "tem_forward" in names and "tem_poles" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(T.EXPORTS)


def test_setup_validation_without_gpu():
    import ctypes as C
    L = T.lib()
    h = C.c_void_p()
    w = np.ones(4)
    p = w.ctypes.data_as(C.POINTER(C.c_double))
    assert L.tem_setup_grid(C.byref(h), 4, 4, 4, p, p, p, 0, 0, None) == T.TEM_EINVAL  # k_surface
    bad = np.array([1.0, -1.0, 1.0, 1.0])
    pb = bad.ctypes.data_as(C.POINTER(C.c_double))
    assert L.tem_setup_grid(C.byref(h), 4, 4, 4, pb, p, p, 2, 0, None) == T.TEM_EINVAL
    assert b"width" in L.tem_last_error(None)
    assert L.tem_setup_grid(C.byref(h), 1, 4, 4, p, p, p, 2, 0, None) == T.TEM_EINVAL
    assert L.tem_forward(None, None, 0, None, 0, 1, 1, None, None, None, None, None, None) == T.TEM_EINVAL


def test_poles_validation():
    with pytest.raises(T.TemError):
        T.poles([1e-3, -1.0], 10)
    with pytest.raises(T.TemError):
        T.poles([1e-3, 1e-2], 1)
    with pytest.raises(T.TemError):
        T.poles([1e-3, np.nan], 10)


TABLE = json.load(open(os.path.join(GOLD, "table1.json")))
COUNTS = json.load(open(os.path.join(GOLD, "paper_counts.json")))


@pytest.mark.parametrize("ratio,tol,m", [(1e3, 1e-6, 27), (1e3, 1e-8, 35), (1e4, 1e-8, 44)])
def test_host_rkfit_table1(ratio, tol, m):
    t = np.logspace(-np.log10(ratio), 0, 31)
    xi, c, err = T.poles(t, m)
    assert err.max() <= 1.2 * tol


def test_host_rkfit_fig1_and_symmetry():
    c = COUNTS
    t = np.logspace(-3, 0, c["fig1_channels"])
    xi, cc, err = T.poles(t, c["fig1_degree"])
    assert len(xi) == c["fig1_pair_count"] and np.all(xi.imag > 0)
    target = complex(*c["fig1_closest_pair"])
    assert np.min(np.abs(xi - target)) / abs(target) < 0.10
    # the family is real on x >= 0: write out both poles of every pair
    x = np.linspace(0, 40, 81)
    full = np.zeros((len(x), len(t)), complex)
    for p, a in zip(xi, cc):
        full += 0.5 * a[None, :] / (x[:, None] - p) + 0.5 * np.conj(a)[None, :] / (x[:, None] - np.conj(p))
    assert np.abs(full.imag).max() <= 1e-12 * np.abs(full.real).max()
    assert np.all(np.abs(np.exp(-np.outer(x, t)) - full.real) <= 1.01 * err[None, :])


def test_host_rkfit_auto_degree_and_scaling():
    t = np.logspace(-6, -2, 40)
    xi, c, err = T.poles(t, 0, tol=1e-8)      # Table 1: ratio 1e4, 1e-8 -> 44
    assert len(xi) >= 22 and err.max() <= 1.2e-8
    xi2, c2, err2 = T.poles(t * 1024.0, 44)
    assert np.allclose(xi2, xi / 1024.0, rtol=1e-12)
    assert np.allclose(err2, err, rtol=1e-9)


def test_host_rkfit_matches_oracle_error_level():
    """Independent implementations of the same reading: the per-channel
    errors agree in order of magnitude (poles need not be identical)."""
    from oracle import rkfit as R
    t = np.logspace(-5, -2, 20)
    xi, c, err = T.poles(t, 38)
    o = R.rkfit(t, 38)
    assert 0.2 < err.max() / o["err"].max() < 5.0


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus N > 1 exits with a message, before any
    GPU work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


@pytest.mark.parametrize("tol,m", list(zip(TABLE["tolerances"], TABLE["degree"]["1"])))
def test_host_single_time_table1(tol, m):
    """tem_poles_single meets Table 1's t_max/t_min = 1 column: degree m
    reaches tol and m - 1 does not."""
    assert T.poles_single(m)[3] <= tol
    assert T.poles_single(m - 1)[3] > tol


def test_host_single_time_best_and_counts():
    """The host fit is the best approximation: its uniform error agrees with
    the oracle's (itself pinned by equioscillation) and lies just below
    Halphen's 2 H^(-m-1/2); conjugate pairs give the 124 and 217 solve counts
    of Sec. 3.1 and 5.1; invalid degrees are refused."""
    from oracle import rkfit, single
    for m in (2, 5, 8, 10):
        xi, a, a0, err = T.poles_single(m)
        fit = {"xi": xi, "alpha": np.where(xi.imag > 0, 0.5, 1.0) * a, "alpha0": a0}
        assert abs(single.uniform_error(fit) - err) <= 1e-6 * err
        assert abs(err - single.best_rational(m)["err"]) <= 1e-3 * err
        assert 0.95 <= err / (2 * rkfit.HALPHEN ** (-m - 0.5)) <= 1.0
        assert np.all((xi.imag > 0) | (xi.real < 0))
    assert 31 * len(T.poles_single(7)[0]) == COUNTS["single_time_m7_K31_solves"]
    assert 31 * len(T.poles_single(14)[0]) == COUNTS["single_time_m14_K31_solves"]
    for m in (0, 33):
        with pytest.raises(T.TemError):
            T.poles_single(m)


def test_forward_single_validation_without_gpu():
    import ctypes as C
    L = T.lib()
    z = np.zeros(4)
    p = z.ctypes.data_as(C.POINTER(C.c_double))
    assert L.tem_forward_single(None, None, 0, None, 0, 1, p, 1, p, p, 0.0, None, None, None, None) == T.TEM_EINVAL
