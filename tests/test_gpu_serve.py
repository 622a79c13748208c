"""Serving loop: continuous admission by HBM footprint, requests overlapping
on the device, and each result identical alone and in the mix."""
import numpy as np
import pytest

import tem_workloads as W
from oracle import rkfit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_11657_amd import tem as T
    T.lib()
    return T


def _requests(n=5):
    from paper_2506_11657_amd.serve import Request
    t = W.log_channels(1e-5, 1e-3, 12)
    reqs = []
    rng = np.random.default_rng(7)
    for i in range(n):
        wl = W.small_case(8 + 2 * (i % 3), seed=100 + i, t=t)
        kind = "adjoint" if i % 2 else "forward"
        r = Request(rid=i, kind=kind, workload=wl, arrival=0.01 * i)
        if kind == "adjoint":
            r.d_obs = np.zeros((1, len(t), len(wl.receivers)))
        reqs.append(r)
    return reqs, t


def test_alone_equals_mix_bitwise(tem):
    from paper_2506_11657_amd.serve import Server, summarize
    reqs, t = _requests()
    fit = rkfit.rkfit(t, 18)
    s, C = rkfit.shifts_and_coefficients(fit)
    alone = Server(-s, C, max_active=1).run(_requests()[0], realtime=False)
    mix_srv = Server(-s, C, max_active=4)
    import time
    t0 = time.perf_counter()
    mix = mix_srv.run(reqs, realtime=True)
    summ = summarize(mix, time.perf_counter() - t0)
    errors = [(r.rid, r.error) for r in mix if r.error is not None]
    assert summ["completed"] == len(reqs), errors
    for a, m in zip(alone, mix):
        assert a.error is None and m.error is None, (a.error, m.error)
        assert np.array_equal(a.data, m.data)
        if a.kind == "adjoint":
            assert np.array_equal(a.grad, m.grad)


def test_admission_by_footprint(tem):
    """A budget that holds one request at a time serializes them; a request
    larger than the budget is rejected without running."""
    from paper_2506_11657_amd.serve import Server, footprint_bytes
    reqs, t = _requests(3)
    fit = rkfit.rkfit(t, 18)
    s, C = rkfit.shifts_and_coefficients(fit)
    fps = [footprint_bytes(len(r.workload.hx), len(r.workload.hy), len(r.workload.hz), len(s), len(r.workload.loops),
                           r.kind, n_rx=len(r.workload.receivers)) for r in reqs]
    srv = Server(-s, C, max_active=8, hbm_budget=max(fps))
    out = srv.run(reqs, realtime=False)
    spans = sorted((r.admitted, r.finished) for r in out)
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0 - 1e-3   # never two requests resident at once
    big = _requests(1)[0]
    srv2 = Server(-s, C, hbm_budget=1 << 20)
    r = srv2.run(big, realtime=False)[0]
    assert r.error is not None and "ENOMEM" in r.error


def _mixed_requests():
    """Forward and adjoint requests on three grid sizes (8^3, 12^3, 16^3), one
    with two loops, and one precision-1 forward (which runs its own launches)."""
    from paper_2506_11657_amd.serve import Request
    t = W.log_channels(1e-5, 1e-3, 12)
    reqs = []
    for i in range(6):
        n = (8, 12, 16)[i % 3]
        wl = W.small_case(n, seed=200 + i, t=t)
        if i == 2:
            wl.loops = [W.Loop(1, n // 2, 1, n // 2, 1.0), W.Loop(n // 2, n - 1, 2, n - 2, -1.5)]
        kind = "adjoint" if i % 2 else "forward"
        r = Request(rid=i, kind=kind, workload=wl, arrival=0.005 * i)
        if kind == "adjoint":
            r.d_obs = np.zeros((len(wl.loops), len(t), len(wl.receivers)))
        if i == 4:
            r.precision = 1
        reqs.append(r)
    return reqs, t


def test_batched_engine_alone_equals_mix_bitwise(tem, monkeypatch):
    """Continuous batching: the FP64 solves of every admitted request run in
    shared batched launches (one stencil and one update launch per iteration
    for all of them).  Requests of different grid sizes share launches (the
    engine saw blocks with several requests' jobs), and every result is
    bitwise the same as the request served alone through the same engine; the
    batched results also agree to rounding with the unbatched path running the
    same two-kernel seed iteration as the engine (TEM_SEED=hs for every
    context of the test, the precision-1 request's own launches included; on
    these small grids the unbatched default is the one-kernel iteration,
    another rounding of CG that the forward tests check against the oracle)."""
    monkeypatch.setenv("TEM_SEED", "hs")
    from paper_2506_11657_amd.serve import Server, summarize
    import time
    reqs, t = _mixed_requests()
    fit = rkfit.rkfit(t, 18)
    s, C = rkfit.shifts_and_coefficients(fit)
    srv_alone = Server(-s, C, max_active=1, batched=True)
    alone = srv_alone.run(_mixed_requests()[0], realtime=False)
    st_alone = srv_alone.engine.stats()
    srv_alone.close()
    srv_mix = Server(-s, C, max_active=4, batched=True)
    t0 = time.perf_counter()
    mix = srv_mix.run(reqs, realtime=True)
    summ = summarize(mix, time.perf_counter() - t0)
    st_mix = srv_mix.engine.stats()
    srv_mix.close()
    print("engine alone:", st_alone, "mix:", st_mix, "summary:", summ)
    errors = [(r.rid, r.error) for r in mix + alone if r.error is not None]
    assert summ["completed"] == len(reqs) and not errors, errors
    assert st_alone["max_contexts"] == 1
    assert st_mix["max_contexts"] >= 2 and st_mix["max_jobs"] >= 2
    for a, m in zip(alone, mix):
        assert np.array_equal(a.data, m.data), a.rid
        if a.kind == "adjoint":
            assert np.array_equal(a.grad, m.grad), a.rid
    # the same requests without the engine, same seed iteration: equal to rounding (other tiles)
    plain = Server(-s, C, max_active=4).run(_mixed_requests()[0], realtime=False)
    for a, p in zip(alone, plain):
        assert p.error is None
        scale = np.abs(p.data).max()
        assert np.abs(a.data - p.data).max() <= 1e-8 * scale, a.rid
        if a.kind == "adjoint":
            assert np.abs(a.grad - p.grad).max() <= 1e-7 * np.abs(p.grad).max(), a.rid
