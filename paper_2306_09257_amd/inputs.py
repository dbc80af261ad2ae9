"""Seeded synthetic problem generators shared by the library tests, the bench
and the oracle checks.

This module describes *problems* (grid, layer rows, channel sets, permittivity
maps, objective weights).  It contains none of the method's arithmetic: no
operator entries, no propagation constants, no solves.  Both the HIP path and
the CPU oracle consume what it returns.

Layer layout (top to bottom, rows of the y axis):
    PML_top (medium eps_top) | eps_top layer | design slab | eps_bot layer | PML_bot (eps_bot)
The source row sits one row below the top PML, the projection row two rows
above the bottom PML.  Channels are the Fourier orders a with |a| < nx*dx/lambda
(the continuum propagating set in air), the same orders on both sides; the
paper's metasurface benchmark counts channels the same way (Supplement Sec. 1,
2W/lambda channels; Sec. 3 for the beam splitter's angular window).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    dx_over_lambda: float
    npml_top: int
    npml_bot: int
    design_row0: int
    design_row1: int
    in_orders: np.ndarray
    out_orders: np.ndarray
    eps_top: float = 1.0
    eps_bot: float = 2.25
    pml_R0: float = 1e-8
    pml_power: int = 3
    src_row: int = -1
    prj_row: int = -1

    def __post_init__(self):
        self.in_orders = np.asarray(self.in_orders, dtype=np.int32)
        self.out_orders = np.asarray(self.out_orders, dtype=np.int32)
        if self.src_row < 0:
            self.src_row = self.npml_top + 1
        if self.prj_row < 0:
            self.prj_row = self.ny - self.npml_bot - 2

    @property
    def n_in(self) -> int:
        return int(self.in_orders.size)

    @property
    def n_out(self) -> int:
        return int(self.out_orders.size)

    @property
    def n_unknowns(self) -> int:
        return self.nx * self.ny

    @property
    def n_design_rows(self) -> int:
        return self.design_row1 - self.design_row0

    @property
    def h(self) -> float:
        """k0*dx, the dimensionless frequency of the dx^2-scaled operator."""
        return 2.0 * math.pi * self.dx_over_lambda

    def background_eps(self) -> np.ndarray:
        """[ny][nx] permittivity with the design rows left at eps_top."""
        eps = np.empty((self.ny, self.nx), dtype=np.float64)
        eps[: self.design_row1, :] = self.eps_top
        eps[self.design_row1:, :] = self.eps_bot
        return eps


def channel_orders(nx: int, dx_over_lambda: float, sin_max: float = 1.0,
                   n_medium: float = 1.0) -> np.ndarray:
    """Orders a with |a| < n_medium * sin_max * nx*dx/lambda (strict)."""
    lim = n_medium * sin_max * nx * dx_over_lambda
    amax = int(math.ceil(lim)) - 1
    while amax + 1 < lim:
        amax += 1
    a = np.arange(-amax, amax + 1, dtype=np.int32)
    return a[np.abs(a) < lim]


def layout_rows(ny: int):
    """(npml, top layer, design, bottom layer, npml) for the row counts used
    by the workloads: 60, 92, 140, 160 (and the pattern for others)."""
    table = {60: (16, 4, 20, 4, 16), 92: (16, 20, 20, 20, 16),
             140: (20, 30, 40, 30, 20), 160: (20, 40, 40, 40, 20)}
    if ny in table:
        return table[ny]
    raise ValueError(f"no layer layout for ny={ny}")


def make_problem(nx: int, ny: int, dx_over_lambda: float = 0.05,
                 layout: Optional[Sequence[int]] = None,
                 in_orders=None, out_orders=None, **kw) -> Problem:
    lay = tuple(layout) if layout is not None else layout_rows(ny)
    if sum(lay) != ny:
        raise ValueError("layout rows must sum to ny")
    npml_t, top, des, bot, npml_b = lay
    d0 = npml_t + top
    if in_orders is None:
        in_orders = channel_orders(nx, dx_over_lambda)
    if out_orders is None:
        out_orders = in_orders
    return Problem(nx=nx, ny=ny, dx_over_lambda=dx_over_lambda,
                   npml_top=npml_t, npml_bot=npml_b, design_row0=d0,
                   design_row1=d0 + des, in_orders=in_orders,
                   out_orders=out_orders, **kw)


# ----------------------------------------------------------------------------
# permittivity maps and objective weights (numpy default_rng, draw order: eps
# first, then w)
# ----------------------------------------------------------------------------

def eps_uniform(prob: Problem, rng: np.random.Generator, lo=1.0, hi=4.0) -> np.ndarray:
    eps = prob.background_eps()
    eps[prob.design_row0:prob.design_row1, :] = rng.uniform(
        lo, hi, size=(prob.n_design_rows, prob.nx))
    return eps


def _gauss_kernel_fwhm(fwhm: float) -> np.ndarray:
    sigma = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    r = int(math.ceil(3.0 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    return k / k.sum()


def eps_binary_smoothed(prob: Problem, rng: np.random.Generator,
                        lo=1.0, hi=4.0, fwhm=3.0) -> np.ndarray:
    """Bernoulli(1/2) pixels over {lo, hi}, then a normalised separable Gaussian
    of the given FWHM: periodic wrap in x, mirror reflection at the slab's y
    edges.  The result stays within [lo, hi]."""
    eps = prob.background_eps()
    nd = prob.n_design_rows
    m = np.where(rng.random((nd, prob.nx)) < 0.5, lo, hi)
    k = _gauss_kernel_fwhm(fwhm)
    r = (k.size - 1) // 2
    # x: periodic
    sm = np.zeros_like(m)
    for t in range(-r, r + 1):
        sm += k[t + r] * np.roll(m, -t, axis=1)
    # y: reflect at the slab edges
    padded = np.pad(sm, ((r, r), (0, 0)), mode="symmetric")
    out = np.zeros_like(sm)
    for t in range(-r, r + 1):
        out += k[t + r] * padded[r + t: r + t + nd, :]
    eps[prob.design_row0:prob.design_row1, :] = np.clip(out, lo, hi)
    return eps


def weights_uniform(prob: Problem, rng: np.random.Generator) -> np.ndarray:
    return rng.uniform(0.0, 1.0, size=(prob.n_out, prob.n_in))


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

def metasurface_small(seed: int = 0):
    """240 x 92 grid (22,080 unknowns), 23 x 23 channels, 4,800 design pixels,
    i.i.d. U[1,4] design permittivity, w ~ U[0,1]."""
    prob = make_problem(240, 92)
    rng = np.random.default_rng(seed)
    eps = eps_uniform(prob, rng)
    w = weights_uniform(prob, rng)
    return prob, eps, w


def metasurface_wide(seed: int = 1, nx: int = 24000):
    """24,000 x 160 grid (3.84M unknowns), 2,399 x 2,399 channels, 960,000
    design pixels: binary {1,4} pixels smoothed by a 3-px-FWHM Gaussian."""
    prob = make_problem(nx, 160)
    rng = np.random.default_rng(seed)
    eps = eps_binary_smoothed(prob, rng)
    w = weights_uniform(prob, rng)
    return prob, eps, w


def batch_uneven(seed: int = 3, count: int = 64, nx_max: int = 4800, nx_step: int = 120):
    """Independent problems of uneven size for one batched factorization: nx
    uniform over {nx_step, 2 nx_step, ..., nx_max}, ny in {60, 92, 140},
    wavelength lambda/lambda0 uniform in [0.9, 1.1] at dx = lambda0/20
    (dx/lambda = 0.05/(lambda/lambda0)), eps ~ U[1, 4] on the design rows,
    w ~ U[0, 1]; channels |a| < nx dx/lambda.  Returns a list of
    (prob, eps, w)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nx = int(rng.integers(1, nx_max // nx_step + 1)) * nx_step
        ny = int(rng.choice([60, 92, 140]))
        lam = float(rng.uniform(0.9, 1.1))
        prob = make_problem(nx, ny, dx_over_lambda=0.05 / lam)
        eps = eps_uniform(prob, rng)
        w = weights_uniform(prob, rng)
        out.append((prob, eps, w))
    return out


def design_loop(seed: int = 4, nx: int = 12000):
    """Differentiation-in-the-loop workload: 12,000 x 140 grid (1.68M unknowns),
    1,199 x 1,199 channels, 480,000 design pixels.  Initial design
    eps = 2.5 + 0.1 N(0,1) clipped to [1, 4]; w ~ U[0,1]."""
    prob = make_problem(nx, 140)
    rng = np.random.default_rng(seed)
    eps = prob.background_eps()
    eps[prob.design_row0:prob.design_row1, :] = np.clip(
        2.5 + 0.1 * rng.standard_normal((prob.n_design_rows, prob.nx)), 1.0, 4.0)
    w = weights_uniform(prob, rng)
    return prob, eps, w


def tiny_problem(nx=24, ny=60, seed=0, layout=None, n_orders=None, **kw):
    """Small grids for oracle pins and parity tests."""
    lay = layout
    if lay is None:
        lay = layout_rows(ny) if ny in (60, 92, 140, 160) else None
    prob = make_problem(nx, ny, layout=lay, **kw)
    if n_orders is not None:
        a = np.arange(-(n_orders // 2), n_orders - n_orders // 2, dtype=np.int32)
        prob.in_orders = a
        prob.out_orders = a
    rng = np.random.default_rng(seed)
    eps = eps_uniform(prob, rng)
    w = weights_uniform(prob, rng)
    return prob, eps, w


# ----------------------------------------------------------------------------
# beam-splitter workload (Sec. 3): period W = 24 um, wavelength 0.94 um,
# a-Si ridges (n = 3.70) of height 0.56 um on silica (n = 1.45) in air, light
# incident from the substrate, inputs |a| < W/(2 lambda) (within +-30 degrees
# in air), outputs |a| < W/lambda (all outgoing orders in air)
# ----------------------------------------------------------------------------

SPLITTER_W_UM = 24.0
SPLITTER_LAMBDA_UM = 0.94
SPLITTER_RIDGE_H_UM = 0.56
SPLITTER_EPS_RIDGE = 3.70 ** 2
SPLITTER_EPS_SUBSTRATE = 1.45 ** 2
SPLITTER_EPS_AIR = 1.0
SPLITTER_MIN_GAP_UM = 0.04


def splitter_problem(nx: int = 1024, npml: int = 20, spacer: int = 12) -> Problem:
    """Grid of one period: nx cells across W, the ridge band rounded to whole
    rows (24 at nx = 1024, dx = 23.4 nm = lambda / 40.1); rows: PML |
    substrate (source side) | ridges | air (projection side) | PML."""
    dx_um = SPLITTER_W_UM / nx
    rows = int(round(SPLITTER_RIDGE_H_UM / dx_um))
    lay = (npml, spacer, rows, spacer, npml)
    dxl = dx_um / SPLITTER_LAMBDA_UM
    return make_problem(nx, sum(lay), dx_over_lambda=dxl, layout=lay,
                        in_orders=channel_orders(nx, dxl, sin_max=0.5),
                        out_orders=channel_orders(nx, dxl),
                        eps_top=SPLITTER_EPS_SUBSTRATE, eps_bot=SPLITTER_EPS_AIR)


def splitter_edges_to_grid(y_um, nx: int) -> np.ndarray:
    """Edge positions y in [-W/2, W/2] (microns, central plane at 0) to grid
    units x = (y / W + 1/2) nx along the periodic axis."""
    return (np.asarray(y_um, dtype=np.float64) / SPLITTER_W_UM + 0.5) * nx


def splitter_random_edges(nx: int, rng: np.random.Generator, n_ridges_half: int = 40) -> np.ndarray:
    """2 n_ridges_half ascending edges of the first half period [0, nx/2] (grid
    units) with every ridge width and gap (the ends included) at least
    40 nm: gaps = minimum + the rest split by a flat Dirichlet draw."""
    n = 2 * n_ridges_half
    half = nx / 2.0
    m = SPLITTER_MIN_GAP_UM / (SPLITTER_W_UM / nx)
    spare = half - (n + 1) * m
    if spare <= 0:
        raise ValueError("grid too coarse for the minimum gap")
    g = m + spare * rng.dirichlet(np.ones(n + 1))
    return np.cumsum(g)[:n]


def beam_splitter(seed: int = 6, nx: int = 1024):
    """The beam-splitter problem with a seeded random initial design:
    (prob, background eps, first-half-period edges in grid units)."""
    prob = splitter_problem(nx)
    rng = np.random.default_rng(seed)
    return prob, prob.background_eps(), splitter_random_edges(nx, rng)


def metasurface_multiangle(seed: int = 2, nx: int = 48000):
    """Multi-angle splitter workload: 48,000 x 160 grid (7.68M unknowns),
    inputs |a| < 0.95 nx dx/lambda (4,559 at nx = 48,000) and the same output
    orders, 1.92M design pixels of binary {1, 4} permittivity smoothed by a
    3-px-FWHM Gaussian.  The objective groups, for each input, the outputs at
    order differences g * delta (|g| <= 2) with delta = nx dx / (24 lambda)
    (a 24-wavelength supercell: 100 orders at nx = 48,000).  Returns
    (prob, eps, delta)."""
    orders = channel_orders(nx, 0.05, sin_max=0.95)
    prob = make_problem(nx, 160, in_orders=orders, out_orders=orders)
    rng = np.random.default_rng(seed)
    eps = eps_binary_smoothed(prob, rng)
    delta = int(round(nx * 0.05 / 24.0))
    return prob, eps, delta
