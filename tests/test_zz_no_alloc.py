"""tem_apply_noalloc (the operator with no device allocation, for callers
that cannot allocate) against tem_apply on the same inputs, through the C ABI:
two calls in a row, the second on a smaller grid, then the first grid again;
both entry points run the same kernels in the same order, so the results are
bitwise equal.  A grid too large for the fixed device array is refused."""
import numpy as np
import pytest

import tem_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_11657_amd import tem as T
    T.lib()
    return T


def _case(tem, wl, seed):
    import torch
    ctx = tem.Context.from_workload(wl)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(ctx.n_storage) + 1j * rng.standard_normal(ctx.n_storage)
    xd = torch.from_numpy(x).to("cuda")
    # stale values in the output must not survive (every entry is written)
    yd = torch.full((ctx.n_storage,), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    return ctx, x, xd, yd


def test_noalloc_apply_matches_apply_bitwise(tem):
    import torch
    big = W.ragged37(1e-5)      # 37 x 10 x 9 cells, several stencil tiles
    small = W.small_case(6, seed=4)
    shifts = [3.5e3 - 2.0e4j, 1e6 + 1e5j]
    c1, x1, x1d, y1d = _case(tem, big, 1)
    c2, x2, x2d, y2d = _case(tem, small, 2)
    for shift in shifts:
        print("noalloc apply: %s grid, shift %r" % (big.name, shift), flush=True)
        c1.apply_noalloc(x1d, y1d, shift)
        torch.cuda.synchronize()
        assert np.array_equal(y1d.cpu().numpy(), c1.apply(x1, shift))
        # second call in a row on a smaller grid: the array holds the first call's data
        print("noalloc apply: %s grid, shift %r" % (small.name, shift), flush=True)
        c2.apply_noalloc(x2d, y2d, shift)
        torch.cuda.synchronize()
        assert np.array_equal(y2d.cpu().numpy(), c2.apply(x2, shift))
    # and the larger grid again after the smaller one
    c1.apply_noalloc(x1d, y1d, shifts[0])
    torch.cuda.synchronize()
    assert np.array_equal(y1d.cpu().numpy(), c1.apply(x1, shifts[0]))
    c1.close()
    c2.close()


def test_noalloc_apply_refuses_oversize_grid(tem):
    import torch
    n = 90   # 91^3 nodes need 2 * 3 * 91^3 * 16 + 256 bytes > 64 MiB
    h = np.full(n, 10.0)
    ctx = tem.Context(h, h, h, n // 2)
    ctx.set_conductivity(np.full((n, n, n), 0.01))
    x = torch.zeros(ctx.n_storage, dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(tem.TemError) as e:
        ctx.apply_noalloc(x, y, 1.0)
    assert e.value.status == tem.TEM_EINVAL and "too large" in str(e.value)
    ctx.close()
