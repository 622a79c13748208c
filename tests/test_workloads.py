"""The seeded synthetic workloads match their stated recipe: grid sizes,
graded widths, air/earth layering, conductivity values, loop and receiver
placement, channel sets and degrees, and they are reproducible from their
seeds.  These are the inputs every parity test and the benchmark run on."""
import numpy as np

import tem_workloads as W


def _geometric(h, ratio, rtol=1e-12):
    return np.allclose(h[1:] / h[:-1], ratio, rtol=rtol)


def test_plain16_recipe():
    wl = W.cfg_plain16()
    assert wl.sigma.shape == (16, 16, 16) and np.all(wl.hx == 20.0) and np.all(wl.hz == 20.0)
    assert wl.k_s == 8 and np.all(wl.sigma[:8] == 0.01) and np.all(wl.sigma[8:] == W.SIGMA_AIR)
    lp = wl.loops[0]
    assert (lp.i1 - lp.i0) * 20.0 == 100.0 and (lp.j1 - lp.j0) * 20.0 == 100.0
    assert len(wl.t) == 20 and np.isclose(wl.t[0], 1e-5) and np.isclose(wl.t[-1], 1e-2)
    assert _geometric(wl.t, (1e-2 / 1e-5) ** (1 / 19), rtol=1e-9) and wl.degree == 38


def test_graded64_recipe():
    wl = W.cfg_graded64()
    assert wl.sigma.shape == (64, 64, 64) and len(wl.hx) == len(wl.hy) == len(wl.hz) == 64
    # 12 core cells of 10 m in x and y, growing x1.1 outwards on both sides
    core = np.where(wl.hx == 10.0)[0]
    assert len(core) == 12 and core[0] == 26 and core[-1] == 37
    assert _geometric(wl.hx[37:], 1.1) and _geometric(wl.hx[:27][::-1], 1.1)
    # 40 earth layers under 24 air layers; 0.1 / 0.01 / 0.05 S/m by depth, plus one 0.5 S/m block
    assert wl.k_s == 40 and np.all(wl.sigma[40:] == W.SIGMA_AIR)
    earth = wl.sigma[:40]
    vals, counts = np.unique(earth, return_counts=True)
    assert set(vals) == {0.01, 0.05, 0.1, 0.5} and counts[list(vals).index(0.5)] == 6 * 6 * 4
    assert np.all(earth[36:][earth[36:] != 0.5] == 0.1) and np.all(earth[28:36][earth[28:36] != 0.5] == 0.01)
    assert np.all(earth[:28][earth[:28] != 0.5] == 0.05)
    lp = wl.loops[0]
    assert np.isclose(np.sum(wl.hx[lp.i0:lp.i1]), 100.0) and np.isclose(np.sum(wl.hy[lp.j0:lp.j1]), 100.0)
    assert wl.receivers == [(32, 32)] and lp.i0 + lp.i1 == 64 and lp.j0 + lp.j1 == 64
    assert len(wl.t) == 40 and np.isclose(wl.t[0], 1e-6) and np.isclose(wl.t[-1], 1e-2) and wl.degree == 44
    # reproducible from its seed, different for another seed (the block moves)
    assert np.array_equal(W.cfg_graded64().sigma, wl.sigma)
    assert not np.array_equal(W.cfg_graded64(seed=2).sigma, wl.sigma)


def test_blocky128_recipe():
    wl = W.cfg_blocky128()
    assert wl.sigma.shape == (128, 128, 128) and wl.k_s == 96
    assert np.all(wl.sigma[96:] == W.SIGMA_AIR)
    ls = np.log10(wl.sigma[:96])
    # constant on 8^3 blocks
    blocks = ls.reshape(12, 8, 16, 8, 16, 8)
    assert np.all(blocks == blocks[:, :1, :, :1, :, :1])
    b = blocks[:, 0, :, 0, :, 0].ravel()
    assert abs(b.mean() + 2.0) < 0.1 and abs(b.std() - 0.7) < 0.1
    assert _geometric(wl.hx[76:], 1.05) and np.sum(wl.hx == 10.0) == 24
    assert np.array_equal(W.cfg_blocky128().sigma, wl.sigma)


def test_serving_trace_recipe():
    tr = W.serving_trace(seed=7, n_req=2000)
    gaps = np.diff([0.0] + [q["arrival"] for q in tr])
    assert abs(gaps.mean() - 1.0 / 200.0) < 0.1 / 200.0            # Poisson at 200 req/s
    assert {q["n"] for q in tr} == {32, 48, 64, 96}
    assert {q["n_src"] for q in tr} == {1, 2, 3, 4}
    kinds = [q["kind"] for q in tr]
    assert 0.45 < kinds.count("forward") / len(kinds) < 0.55
    assert W.serving_trace(seed=7, n_req=2000) == tr
    wl = W.serving_request(48, 3, tr[0]["seed"])
    assert wl.sigma.shape == (48, 48, 48) and len(wl.loops) == 3
    # 12-cell 10 m core, growth 1.1**(64/n): extents 0.78, 1.6, 2.5 (the 64^3
    # benchmark grid's) and 4.5 km
    ext = {n: np.sum(W.serving_request(n, 1, 5).hx) for n in (32, 48, 64, 96)}
    assert np.isclose(ext[64], np.sum(W.cfg_graded64().hx))
    assert np.allclose([ext[32], ext[48], ext[96]], [780.0, 1603.1, 4480.0], rtol=1e-3)
    for n in (32, 48, 96):
        hx = W.serving_request(n, 1, 5).hx
        assert np.sum(hx == 10.0) == 12 and _geometric(hx[(n + 12) // 2:], 1.1 ** (64.0 / n))
