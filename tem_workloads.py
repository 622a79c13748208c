"""Seeded synthetic TEM workloads shared by the oracle and the HIP path.

This module only builds inputs: cell widths, per-cell conductivity, loop
sources, receivers and channel times.  It holds none of the method's
arithmetic (no operators, no poles, no solves), so that the oracle and the
HIP library can both take their inputs from here without sharing any code
of the computation itself.

Conventions (shared by every consumer):
  * cells are indexed (i, j, k) with x fastest; k = 0 is the bottom layer and
    z points up; ``sigma`` has shape (Nz, Ny, Nx);
  * the ground surface z = 0 is node plane ``k_s``: cells k < k_s are earth,
    cells k >= k_s are air;
  * a loop is given by node indices (i0, i1, j0, j1) in the plane k_s and
    runs counter-clockwise seen from +z with current ``current`` [A];
  * a receiver is the surface z-face of cell column (i, j) in plane k_s.

The physical set-up follows the paper's test model (Sec. 5: a loop at the
air/earth interface, air of 1e-8 S/m, dB_z/dt at the loop centre) at the
sizes of the benchmark configurations; the paper's own mesh and data are not
available, so every config here is synthetic and seeded.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SIGMA_AIR = 1e-8  # S/m, as in the paper's test model (Sec. 5)


@dataclass
class Loop:
    i0: int
    i1: int
    j0: int
    j1: int
    current: float = 1.0


@dataclass
class Workload:
    name: str
    hx: np.ndarray
    hy: np.ndarray
    hz: np.ndarray
    k_s: int
    sigma: np.ndarray  # (Nz, Ny, Nx) S/m
    loops: list = field(default_factory=list)
    receivers: list = field(default_factory=list)  # list of (i, j) surface z-faces
    t: np.ndarray = None  # channel times [s]
    degree: int = 0  # RKFIT degree (m-hat) proposed for this channel set

    @property
    def shape(self):
        return (len(self.hz), len(self.hy), len(self.hx))

    def node_coords(self):
        """Node coordinates with z = 0 at plane k_s and x, y = 0 at the domain centre."""
        x = np.concatenate([[0.0], np.cumsum(self.hx)])
        y = np.concatenate([[0.0], np.cumsum(self.hy)])
        z = np.concatenate([[0.0], np.cumsum(self.hz)])
        return x - x[-1] / 2, y - y[-1] / 2, z - z[self.k_s]


def log_channels(t0: float, t1: float, n: int) -> np.ndarray:
    """n log-spaced channel times in [t0, t1]."""
    return 10.0 ** np.linspace(np.log10(t0), np.log10(t1), n)


def graded_axis(core_cells: int, h0: float, side_cells: int, growth: float) -> np.ndarray:
    """Widths: a uniform core of ``core_cells`` x h0, then ``side_cells`` cells
    on each side growing geometrically by ``growth`` (h0*growth**p, p = 1..)."""
    side = h0 * growth ** np.arange(1, side_cells + 1)
    return np.concatenate([side[::-1], np.full(core_cells, h0), side])


def graded_z(n_air: int, n_earth: int, h0: float, growth: float) -> np.ndarray:
    """Vertical widths bottom->top: earth cells growing with depth, air cells
    growing with height, both h0 at the surface."""
    earth = h0 * growth ** np.arange(n_earth)
    air = h0 * growth ** np.arange(n_air)
    return np.concatenate([earth[::-1], air])


def centred_loop(n: int, cells: int, current: float = 1.0) -> Loop:
    """Square loop of ``cells`` x ``cells`` cells centred on node n//2 (n even)."""
    c = n // 2
    return Loop(c - cells // 2, c + cells - cells // 2, c - cells // 2, c + cells - cells // 2, current)


def blocky_log_sigma(shape, block: int, mean: float, std: float, rng) -> np.ndarray:
    """log10 sigma constant on block^3 cell blocks aligned to multiples of ``block``."""
    nz, ny, nx = shape
    bz, by, bx = -(-nz // block), -(-ny // block), -(-nx // block)
    v = rng.normal(mean, std, size=(bz, by, bx))
    v = np.repeat(np.repeat(np.repeat(v, block, 0), block, 1), block, 2)[:nz, :ny, :nx]
    return v


# ---------------------------------------------------------------------------
# Benchmark configurations (sizes from the benchmark list; geometry filled in)
# ---------------------------------------------------------------------------

def cfg_plain16() -> Workload:
    """16^3 uniform 20 m grid, 8 air layers (1e-8 S/m) over an 8-layer
    0.01 S/m half-space, 100 m loop on the surface, receiver at its centre,
    20 channels in [1e-5, 1e-2] s.  Deterministic."""
    n = 16
    h = np.full(n, 20.0)
    sigma = np.full((n, n, n), SIGMA_AIR)
    sigma[:8] = 0.01
    return Workload("plain16", h, h.copy(), h.copy(), 8, sigma,
                    loops=[Loop(6, 11, 6, 11, 1.0)], receivers=[(8, 8)],
                    t=log_channels(1e-5, 1e-2, 20), degree=38)


def cfg_graded64(seed: int = 1) -> Workload:
    """64^3 graded grid (10 m core around the loop, x1.1 growth to the
    boundary), three-layer earth (0.1 / 0.01 / 0.05 S/m) with a seeded
    0.5 S/m 6x6x4 block, 100 m centred loop, 40 channels in [1e-6, 1e-2] s."""
    rng = np.random.default_rng(seed)
    hx = graded_axis(12, 10.0, 26, 1.1)
    hz = graded_z(24, 40, 10.0, 1.1)
    n_earth = 40
    sigma = np.full((64, 64, 64), SIGMA_AIR)
    for k in range(n_earth):
        d = n_earth - 1 - k  # earth cell index below the surface
        sigma[k] = 0.1 if d <= 3 else (0.01 if d <= 11 else 0.05)
    core0 = 26
    bx = int(rng.integers(core0 - 10, core0 + 12 + 10 - 6 + 1))
    by = int(rng.integers(core0 - 10, core0 + 12 + 10 - 6 + 1))
    bd = int(rng.integers(2, 10 + 1))
    k_top = n_earth - 1 - bd
    sigma[k_top - 3:k_top + 1, by:by + 6, bx:bx + 6] = 0.5
    return Workload("graded64", hx, hx.copy(), hz, n_earth, sigma,
                    loops=[centred_loop(64, 10)], receivers=[(32, 32)],
                    t=log_channels(1e-6, 1e-2, 40), degree=44)


def cfg_blocky128(seed: int = 2) -> Workload:
    """128^3 graded grid (growth 1.05), 32 air layers, blocky log-normal earth
    (8^3 blocks, log10 sigma ~ N(-2, 0.7)), 100 m centred loop, 40 channels."""
    rng = np.random.default_rng(seed)
    hx = graded_axis(24, 10.0, 52, 1.05)
    hz = graded_z(32, 96, 10.0, 1.05)
    sigma = np.full((128, 128, 128), SIGMA_AIR)
    ls = blocky_log_sigma((96, 128, 128), 8, -2.0, 0.7, rng)
    sigma[:96] = 10.0 ** ls
    return Workload("blocky128", hx, hx.copy(), hz, 96, sigma,
                    loops=[centred_loop(128, 10)], receivers=[(64, 64)],
                    t=log_channels(1e-6, 1e-2, 40), degree=44)


def surface_receivers(n: int, hx: np.ndarray, count: int, radius: float, rng, exclude=()) -> list:
    """``count`` distinct surface z-faces whose centres lie within ``radius``
    of the domain centre (x and y each)."""
    xc = np.concatenate([[0.0], np.cumsum(hx)])
    mid = 0.5 * (xc[:-1] + xc[1:]) - xc[-1] / 2
    ok = np.where(np.abs(mid) <= radius)[0]
    cand = [(int(i), int(j)) for j in ok for i in ok if (int(i), int(j)) not in exclude]
    pick = rng.choice(len(cand), size=count, replace=False)
    return [cand[p] for p in sorted(pick)]


def cfg_inverse(n: int = 64, seed_true: int = 3, seed_cur: int = 4, seed_rx: int = 5,
                n_rx: int = 30, block: int = 8, n_t: int = 40) -> tuple:
    """Differentiation workload: a true and a current blocky log-conductivity
    model on the graded grid (n = 64) or the uniform 20 m grid (n = 16, 4^3
    blocks), 30 surface receivers near the loop, 40 channels.  Returns
    (true_workload, current_workload)."""
    if n == 64:
        hx = graded_axis(12, 10.0, 26, 1.1)
        hz = graded_z(24, 40, 10.0, 1.1)
        n_earth, radius, loop = 40, 200.0, centred_loop(64, 10)
    elif n == 16:
        hx = np.full(16, 20.0)
        hz = np.full(16, 20.0)
        n_earth, radius, loop = 8, 100.0, Loop(6, 11, 6, 11, 1.0)
        block = 4
    else:
        raise ValueError("n must be 16 or 64")
    rx = surface_receivers(n, hx, n_rx, radius, np.random.default_rng(seed_rx))
    models = []
    for seed in (seed_true, seed_cur):
        rng = np.random.default_rng(seed)
        sigma = np.full((n, n, n), SIGMA_AIR)
        sigma[:n_earth] = 10.0 ** blocky_log_sigma((n_earth, n, n), block, -2.0, 0.7, rng)
        models.append(Workload("inverse%d" % n, hx, hx.copy(), hz, n_earth, sigma,
                               loops=[loop], receivers=list(rx),
                               t=log_channels(1e-6, 1e-2, n_t), degree=44))
    return models[0], models[1]


def small_case(n: int = 6, seed: int = 0, n_air: int = None, h: float = 20.0,
               loop: Loop = None, t=None, sigma_air: float = SIGMA_AIR) -> Workload:
    """A tiny uniform grid with random earth conductivity, for dense checks."""
    rng = np.random.default_rng(seed)
    n_air = n // 2 if n_air is None else n_air
    n_earth = n - n_air
    sigma = np.full((n, n, n), sigma_air)
    sigma[:n_earth] = 10.0 ** rng.uniform(-2.5, -0.5, size=(n_earth, n, n))
    hs = np.full(n, h)
    if loop is None:
        loop = Loop(1, n - 1, 1, n - 1, 1.0)
    if t is None:
        t = log_channels(1e-5, 1e-3, 12)
    return Workload("small%d" % n, hs, hs.copy(), hs.copy(), n_earth, sigma,
                    loops=[loop], receivers=[(n // 2 - 1, n // 2 - 1)], t=np.asarray(t), degree=28)


def serving_trace(seed: int = 7, n_req: int = 400, rate: float = 200.0) -> list:
    """Poisson arrivals of forward/adjoint requests on grids of 32..96 cells."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for r in range(n_req):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice([32, 48, 64, 96]))
        out.append({"arrival": t, "kind": "forward" if rng.random() < 0.5 else "adjoint",
                    "n": n, "n_src": int(rng.integers(1, 5)), "seed": int(rng.integers(0, 2**31 - 1))})
    return out


def serving_request(n: int, n_src: int, seed: int) -> Workload:
    """One serving request: graded grid of n cells per axis, a 12-cell 10 m
    core and growth 1.1**(64/n) outwards (horizontal extent 0.78 km at n = 32,
    1.6 km at 48, 2.5 km at 64 as the 64^3 benchmark grid, 4.5 km at 96),
    blocky conductivity, n_src loops of 100 m at distinct seeded surface
    positions in the core."""
    rng = np.random.default_rng(seed)
    g = 1.1 ** (64.0 / n)
    core = 12
    side = (n - core) // 2
    hx = graded_axis(core, 10.0, side, g)
    n_air = (3 * n) // 8
    n_earth = n - n_air
    hz = graded_z(n_air, n_earth, 10.0, g)
    sigma = np.full((n, n, n), SIGMA_AIR)
    sigma[:n_earth] = 10.0 ** blocky_log_sigma((n_earth, n, n), 8, -2.0, 0.7, rng)
    loops = []
    used = set()
    c0 = side
    while len(loops) < n_src:
        i0 = int(rng.integers(c0 - 4, c0 + 4))
        j0 = int(rng.integers(c0 - 4, c0 + 4))
        if (i0, j0) in used:
            continue
        used.add((i0, j0))
        loops.append(Loop(i0, i0 + 10, j0, j0 + 10, 1.0))
    return Workload("serve%d" % n, hx, hx.copy(), hz, n_earth, sigma, loops=loops,
                    receivers=[(n // 2, n // 2)], t=log_channels(1e-6, 1e-2, 40), degree=44)


# ---------------------------------------------------------------------------
# Ragged multi-tile test grids (random widths, several stencil tiles with
# partial tails in x, y and z); shared by the oracle's floor measurement and
# the GPU parity tests
# ---------------------------------------------------------------------------

def ragged37(sigma_air: float = SIGMA_AIR) -> Workload:
    """37 x 10 x 9 cells of 8-25 m, random earth in the bottom 5 layers, two
    loops (1 A and 2.5 A), three receivers, 12 channels in [1e-5, 1e-3] s."""
    rng = np.random.default_rng(3)
    hx, hy, hz = rng.uniform(8, 25, 37), rng.uniform(8, 25, 10), rng.uniform(8, 25, 9)
    sigma = np.full((9, 10, 37), sigma_air)
    sigma[:5] = 10 ** rng.uniform(-2.5, -0.5, (5, 10, 37))
    return Workload("ragged37", hx, hy, hz, 5, sigma,
                    loops=[Loop(3, 12, 2, 7, 1.0), Loop(20, 33, 3, 8, 2.5)],
                    receivers=[(7, 4), (25, 5), (30, 1)], t=log_channels(1e-5, 1e-3, 12), degree=16)


def ragged70(sigma_air: float = 1e-5) -> Workload:
    """70 x 11 x 9 cells of 8-25 m (odd nz: a two-plane stencil tile holds one
    plane at the top), random earth in the bottom 5 layers, one loop, two
    receivers, 10 channels in [1e-5, 1e-3] s."""
    rng = np.random.default_rng(21)
    hx, hy, hz = rng.uniform(8, 25, 70), rng.uniform(8, 25, 11), rng.uniform(8, 25, 9)
    sigma = np.full((9, 11, 70), sigma_air)
    sigma[:5] = 10 ** rng.uniform(-2.5, -0.5, (5, 11, 70))
    return Workload("ragged70", hx, hy, hz, 5, sigma, loops=[Loop(10, 40, 2, 8, 1.0)],
                    receivers=[(25, 5), (60, 3)], t=log_channels(1e-5, 1e-3, 10), degree=16)


def ragged29(sigma_air: float = SIGMA_AIR) -> Workload:
    """29 x 13 x 10 cells of 8-25 m, random earth in the bottom 6 layers, two
    loops (1 A and -2 A), two receivers, 12 channels in [1e-5, 1e-3] s."""
    rng = np.random.default_rng(11)
    hx, hy, hz = rng.uniform(8, 25, 29), rng.uniform(8, 25, 13), rng.uniform(8, 25, 10)
    sigma = np.full((10, 13, 29), sigma_air)
    sigma[:6] = 10 ** rng.uniform(-2.5, -0.5, (6, 13, 29))
    return Workload("ragged29", hx, hy, hz, 6, sigma,
                    loops=[Loop(3, 12, 2, 9, 1.0), Loop(15, 26, 4, 10, -2.0)],
                    receivers=[(7, 5), (20, 6)], t=log_channels(1e-5, 1e-3, 12), degree=16)
