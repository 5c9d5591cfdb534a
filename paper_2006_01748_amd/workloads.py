"""Seeded synthetic inputs for the Gatenby-Gawlinski finite-volume step.

This module only *draws* inputs: initial states, diffusion-tensor fields given by
their eigen-description (lambda1, lambda2, theta), or by (a, b, c) directly, reaction
parameters and run lengths.  It holds none of the scheme's arithmetic: no stencil,
no tensor rotation, no time-step rule.  Both the CPU oracle and the HIP library
consume what it returns, and each side does its own arithmetic on it.

The model (Section 1, eq. (1)) has normal cells u, tumour cells v and excess lactic
acid w on the unit square with Neumann boundaries; the acid diffuses with a
symmetric positive-definite, heterogeneous tensor A = [[a, b], [b, c]] (eq. (2)).
The paper prints no initial data or parameters for its runs, so the workloads
below are synthetic and stand in for "tissue-like" anisotropic media:

* ``cfg0`` 128x128, isotropic A = I, one central tumour disk (radius 0.1).
* ``cfg1`` 1024x1024, smooth random orientation and anisotropy, five disks.
* ``cfg2`` 4096x4096 layered tissue: 64 Voronoi regions with piecewise-constant
  tensors and thin low-diffusion membranes along region borders.
* ``cfg3`` ensembles of uneven square instances (64..512) with per-instance
  parameters.
* ``cfg4`` 512x512 smooth anisotropic field for gradient runs.
* ``tissue3`` 256^3 three-dimensional slab tissue (the model is stated for
  dimension 2 or 3): eight z-slabs of piecewise-constant random SPD tensors with
  a per-cell perturbation, one central tumour ball.

Every random draw uses ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BASE_SEED = 2006017480

# Reaction parameters in the order (delta1, rho2, Delta2, rho3, delta3).  The paper
# writes d, r, alpha and c (eq. (1)); delta1 = d, rho2 = r, Delta2 = alpha and the
# acid term c(V - W) is generalised to rho3 V - delta3 W.
PARAMS_REF = (12.5, 1.0, 0.01, 70.0, 70.0)


@dataclasses.dataclass
class Workload:
    """One synthetic run: grid, tensor description, initial state, parameters."""

    name: str
    nx: int
    ny: int
    lx: float
    ly: float
    params: tuple                 # (delta1, rho2, Delta2, rho3, delta3)
    u0: np.ndarray                # (ny, nx) float64, row-major, x fastest
    v0: np.ndarray
    w0: np.ndarray
    # exactly one of the two tensor descriptions is set
    abc: Optional[tuple] = None   # (a, b, c) arrays
    eig: Optional[tuple] = None   # (lambda1, lambda2, theta) arrays
    safety: float = 0.9           # fraction of the explicit stability bound
    steps: int = 1
    seed: int = 0
    dt_closed_form: Optional[float] = None   # only where the recipe states dt outright
    mass_every: int = 0

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def cell_centres(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0):
    """Cell-centre coordinates ((i + 1/2) dx, (j + 1/2) dy) as (ny, nx) arrays."""
    x = (np.arange(nx, dtype=np.float64) + 0.5) * (lx / nx)
    y = (np.arange(ny, dtype=np.float64) + 0.5) * (ly / ny)
    return np.meshgrid(x, y)  # X[j, i], Y[j, i]


def smooth_field(rng: np.random.Generator, nx: int, ny: int, modes: int = 16,
                 kmin: int = 1, kmax: int = 8) -> np.ndarray:
    """Sum of ``modes`` plane cosines with integer wavenumbers in [kmin, kmax],
    uniform directions and phases, min-max normalised to [0, 1]."""
    X, Y = cell_centres(nx, ny)
    kappa = rng.integers(kmin, kmax + 1, size=modes)
    psi = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    S = np.zeros((ny, nx))
    for m in range(modes):
        S += np.cos(2.0 * math.pi * kappa[m] * (X * math.cos(psi[m]) + Y * math.sin(psi[m]))
                    + phi[m])
    lo, hi = S.min(), S.max()
    return (S - lo) / (hi - lo)


def disks_state(nx: int, ny: int, centres, radius: float):
    """u = 1, v = 0, w = 0 outside; u = 0, v = 1 inside disks (cell centre test)."""
    X, Y = cell_centres(nx, ny)
    inside = np.zeros((ny, nx), dtype=bool)
    for (x0, y0) in centres:
        inside |= (X - x0) ** 2 + (Y - y0) ** 2 <= radius * radius
    u = np.where(inside, 0.0, 1.0)
    v = np.where(inside, 1.0, 0.0)
    w = np.zeros((ny, nx))
    return u, v, w


def smooth_eig_fields(rng: np.random.Generator, nx: int, ny: int,
                      lam_lo: float = 0.5, lam_hi: float = 2.0, ratio_max: float = 10.0):
    """theta = pi * S1, anisotropy ratio = 1 + (ratio_max - 1) * S2, lambda1 i.i.d.
    uniform per cell, lambda2 = lambda1 / ratio."""
    theta = math.pi * smooth_field(rng, nx, ny)
    ratio = 1.0 + (ratio_max - 1.0) * smooth_field(rng, nx, ny)
    lam1 = rng.uniform(lam_lo, lam_hi, size=(ny, nx))
    lam2 = lam1 / ratio
    return lam1, lam2, theta


def voronoi_labels(rng: np.random.Generator, nx: int, ny: int, nseeds: int = 64) -> np.ndarray:
    """Nearest-seed labels of cell centres (ties go to the lower seed index: a
    later seed replaces the running best only when strictly closer)."""
    seeds = rng.uniform(0.0, 1.0, size=(nseeds, 2))
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    best = np.full((ny, nx), np.inf)
    labels = np.zeros((ny, nx), dtype=np.int32)
    d = np.empty((ny, nx))
    for s in range(nseeds):
        np.add(((y - seeds[s, 1]) ** 2)[:, None], ((x - seeds[s, 0]) ** 2)[None, :], out=d)
        closer = d < best
        np.copyto(best, d, where=closer)
        labels[closer] = s
    return labels


def membrane_mask(labels: np.ndarray) -> np.ndarray:
    """A cell is membrane if any 4-neighbour lies in another region (two cells
    wide across every border)."""
    m = np.zeros(labels.shape, dtype=bool)
    d = labels[:, 1:] != labels[:, :-1]
    m[:, 1:] |= d
    m[:, :-1] |= d
    d = labels[1:, :] != labels[:-1, :]
    m[1:, :] |= d
    m[:-1, :] |= d
    return m


def layered_eig_fields(rng: np.random.Generator, nx: int, ny: int, nregions: int = 64,
                       membrane_scale: float = 0.05):
    """Piecewise-constant (lambda1, lambda2, theta) on Voronoi regions, with both
    eigenvalues scaled by ``membrane_scale`` on membrane cells."""
    labels = voronoi_labels(rng, nx, ny, nregions)
    th_r = rng.uniform(0.0, math.pi, size=nregions)
    l1_r = rng.uniform(0.2, 2.0, size=nregions)
    ratio_r = rng.uniform(1.0, 20.0, size=nregions)
    theta = th_r[labels]
    lam1 = l1_r[labels]
    lam2 = lam1 / ratio_r[labels]
    mem = membrane_mask(labels)
    lam1 = np.where(mem, lam1 * membrane_scale, lam1)
    lam2 = np.where(mem, lam2 * membrane_scale, lam2)
    return lam1, lam2, theta


# ---------------------------------------------------------------------------
# The five standard workloads


def cfg0(seed: int = BASE_SEED + 0, n: int = 128, steps: int = 2000) -> Workload:
    """128^2, isotropic A = I, central disk r = 0.1; dt = 0.2 h^2 / (4 max(1, Delta2))."""
    u, v, w = disks_state(n, n, [(0.5, 0.5)], 0.1)
    ones, zeros = np.ones((n, n)), np.zeros((n, n))
    h = 1.0 / n
    dt = 0.2 * h * h / (4.0 * max(1.0, PARAMS_REF[2]))
    return Workload("cfg0", n, n, 1.0, 1.0, PARAMS_REF, u, v, w, abc=(ones, zeros, ones.copy()),
                    safety=0.2, steps=steps, seed=seed, dt_closed_form=dt)


def cfg1(seed: int = BASE_SEED + 1, n: int = 1024, steps: int = 20000) -> Workload:
    """Smooth anisotropic heterogeneous tensor, five disks r = 0.03."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam1, lam2, theta = smooth_eig_fields(rng, n, n)
    centres = rng.uniform(0.1, 0.9, size=(5, 2))
    u, v, w = disks_state(n, n, centres, 0.03)
    return Workload("cfg1", n, n, 1.0, 1.0, PARAMS_REF, u, v, w, eig=(lam1, lam2, theta),
                    safety=0.9, steps=steps, seed=seed)


def cfg2(seed: int = BASE_SEED + 2, n: int = 4096, delta1: float = 12.5,
         steps: int = 10000) -> Workload:
    """Layered tissue: Voronoi regions with membranes, central disk r = 0.05."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam1, lam2, theta = layered_eig_fields(rng, n, n)
    u, v, w = disks_state(n, n, [(0.5, 0.5)], 0.05)
    p = (delta1,) + PARAMS_REF[1:]
    return Workload("cfg2", n, n, 1.0, 1.0, p, u, v, w, eig=(lam1, lam2, theta),
                    safety=0.9, steps=steps, seed=seed, mass_every=500)


CFG3_SIDES = tuple(range(64, 513, 32))


def cfg3_instance(i: int, steps: int = 5000, side: Optional[int] = None) -> Workload:
    """Instance i of the ensemble: own size, parameters, tensor and dt."""
    seed = BASE_SEED + 1000 + i
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.choice(CFG3_SIDES)) if side is None else int(side)
    delta1 = rng.uniform(0.5, 20.0)
    Delta2 = 10.0 ** rng.uniform(-4.0, -1.0)
    r3 = rng.uniform(10.0, 100.0)
    lam1, lam2, theta = smooth_eig_fields(rng, n, n)
    u, v, w = disks_state(n, n, [(0.5, 0.5)], 0.1)
    return Workload(f"cfg3[{i}]", n, n, 1.0, 1.0, (delta1, 1.0, Delta2, r3, r3), u, v, w,
                    eig=(lam1, lam2, theta), safety=0.9, steps=steps, seed=seed)


def cfg3(count: int = 256, steps: int = 5000):
    return [cfg3_instance(i, steps) for i in range(count)]


def cfg4(seed: int = BASE_SEED + 4, n: int = 512, steps: int = 5000) -> Workload:
    """Smooth anisotropic tensor (true theta), five disks r = 0.03, true parameters."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam1, lam2, theta = smooth_eig_fields(rng, n, n)
    centres = rng.uniform(0.1, 0.9, size=(5, 2))
    u, v, w = disks_state(n, n, centres, 0.03)
    return Workload("cfg4", n, n, 1.0, 1.0, PARAMS_REF, u, v, w, eig=(lam1, lam2, theta),
                    safety=0.9, steps=steps, seed=seed)


def cfg4_perturbation(seed: int = BASE_SEED + 4, n: int = 512):
    """Perturbed parameters (each scaled by 1 +/- 0.2, seeded signs) and a theta
    perturbation 0.1 pi * S with S a fresh smooth field mapped to [-1, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed + 500))
    signs = rng.choice([-1.0, 1.0], size=5)
    p = tuple(PARAMS_REF[k] * (1.0 + 0.2 * signs[k]) for k in range(5))
    dtheta = 0.1 * math.pi * (2.0 * smooth_field(rng, n, n) - 1.0)
    return p, dtheta


def front_instance(delta1: float, kappa: float, nx: int = 512, ny: int = 256, lx: float = 1.0,
                   ly: float = 0.5, steps: int = 0, seed: int = BASE_SEED + 5, Delta2: float = 0.01) -> Workload:
    """Propagating-front workload (Section 2's invasion experiment): healthy
    tissue u = 1 everywhere, the tumour v = 1 behind a front at x0(y) = 0.2 +
    0.02 sin(4 pi y / ly + phase) (seeded phase), no acid.  The fronts advance
    along +x.  The acid diffuses with kappa * lam along x, the direction of
    propagation (lower diffusivity there for kappa < 1), and lam across it, lam a
    smooth seeded field in [0.75, 1.25] (heterogeneous); as (lambda1, lambda2,
    theta) = (kappa lam, lam, 0).  Parameters (delta1, 1, Delta2, 70, 70), Delta2 =
    0.01 unless given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = cell_centres(nx, ny, lx, ly)
    phase = rng.uniform(0.0, 2.0 * math.pi)
    x0 = 0.2 + 0.02 * np.sin(4.0 * math.pi * Y / ly + phase)
    v = (X < x0).astype(np.float64)
    u = np.ones((ny, nx))
    w = np.zeros((ny, nx))
    lam = 0.75 + 0.5 * smooth_field(rng, nx, ny)
    theta = np.zeros((ny, nx))
    return Workload(f"front d={delta1} kappa={kappa} D2={Delta2}", nx, ny, lx, ly, (delta1, 1.0, Delta2, 70.0, 70.0),
                    u, v, w, eig=(kappa * lam, lam, theta), safety=0.9, steps=steps, seed=seed)


def front_sweep(deltas=(0.5, 0.8, 1.5, 3.0, 6.0, 12.5), kappas=(1.0, 0.2), nx: int = 512, ny: int = 256,
                steps: int = 0):
    """The delta1 sweep across 1 for each ratio kappa of the acid diffusivity
    along the propagation direction to the one across it: one front_instance
    per (delta1, kappa), all with the same seeded front and heterogeneity."""
    return [front_instance(d, k, nx, ny, steps=steps) for k in kappas for d in deltas]


def random_state(rng: np.random.Generator, nx: int, ny: int):
    """Generic smooth-plus-noise state in [0, 1] for operator tests."""
    u = rng.uniform(0.0, 1.0, size=(ny, nx))
    v = rng.uniform(0.0, 1.0, size=(ny, nx))
    w = rng.uniform(0.0, 1.0, size=(ny, nx))
    return u, v, w


def random_eig(rng: np.random.Generator, nx: int, ny: int, ratio_max: float = 10.0):
    """Per-cell random SPD tensor in eigen form (rough, not smooth)."""
    lam1 = rng.uniform(0.5, 2.0, size=(ny, nx))
    lam2 = lam1 / rng.uniform(1.0, ratio_max, size=(ny, nx))
    theta = rng.uniform(0.0, math.pi, size=(ny, nx))
    return lam1, lam2, theta


def random_abc(rng: np.random.Generator, nx: int, ny: int):
    """Per-cell random SPD tensor drawn directly as (a, b, c): a, c uniform in
    [0.5, 2], b = r sqrt(a c) with |r| < 0.9, so a c - b^2 > 0."""
    a = rng.uniform(0.5, 2.0, size=(ny, nx))
    c = rng.uniform(0.5, 2.0, size=(ny, nx))
    b = rng.uniform(-0.9, 0.9, size=(ny, nx)) * np.sqrt(a * c)
    return a, b, c


def random_tensor3(rng: np.random.Generator, nx: int, ny: int, nz: int, corr: float = 0.45):
    """Per-cell random SPD 3x3 tensor (axx, ayy, azz, axy, axz, ayz): diagonal
    uniform in [0.5, 2], off-diagonal a_ij = r sqrt(a_ii a_jj) with |r| < corr.
    The correlation matrix has unit diagonal and off-diagonals below corr in
    magnitude, so for corr < 1/2 it (hence the tensor) is positive definite."""
    shape = (nz, ny, nx)
    axx, ayy, azz = (rng.uniform(0.5, 2.0, size=shape) for _ in range(3))
    axy = rng.uniform(-corr, corr, size=shape) * np.sqrt(axx * ayy)
    axz = rng.uniform(-corr, corr, size=shape) * np.sqrt(axx * azz)
    ayz = rng.uniform(-corr, corr, size=shape) * np.sqrt(ayy * azz)
    return axx, ayy, azz, axy, axz, ayz


def random_state3(rng: np.random.Generator, nx: int, ny: int, nz: int):
    """Uniform [0, 1] state (u, v, w) of shape (nz, ny, nx) for operator tests."""
    return tuple(rng.uniform(0.0, 1.0, size=(nz, ny, nx)) for _ in range(3))


@dataclasses.dataclass
class Workload3:
    """One synthetic three-dimensional run."""

    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    params: tuple
    u0: np.ndarray                # (nz, ny, nx) float64, x fastest
    v0: np.ndarray
    w0: np.ndarray
    tensor: tuple                 # (axx, ayy, azz, axy, axz, ayz)
    safety: float = 0.9
    steps: int = 1
    seed: int = 0

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


def tissue3(seed: int = BASE_SEED + 30, n: int = 256, nz: Optional[int] = None, steps: int = 100,
            slabs: int = 8) -> Workload3:
    """Three-dimensional slab tissue on the unit cube: ``slabs`` layers along z,
    each with one random SPD tensor (random_tensor3 of a single cell), every cell
    scaled by a factor uniform in [0.9, 1.1]; a tumour ball of radius 0.15 at the
    centre (v = 1, u = 0 inside; u = 1, v = 0 outside), no acid.  Parameters
    PARAMS_REF."""
    nz = n if nz is None else nz
    rng = np.random.Generator(np.random.PCG64(seed))
    slab = [random_tensor3(rng, 1, 1, 1) for _ in range(slabs)]
    layer = np.minimum((np.arange(nz) * slabs) // nz, slabs - 1)
    scale = rng.uniform(0.9, 1.1, size=(nz, n, n))
    tensor = tuple(np.ascontiguousarray(np.array([slab[layer[k]][q][0, 0, 0] for k in range(nz)])[:, None, None]
                                        * scale) for q in range(6))
    x = (np.arange(n) + 0.5) / n
    z = (np.arange(nz) + 0.5) / nz
    r2 = (x[None, None, :] - 0.5) ** 2 + (x[None, :, None] - 0.5) ** 2 + (z[:, None, None] - 0.5) ** 2
    v = (r2 < 0.15 ** 2).astype(np.float64)
    u = 1.0 - v
    w = np.zeros_like(v)
    return Workload3(f"tissue3 {n}x{n}x{nz}", n, n, nz, 1.0, 1.0, 1.0, PARAMS_REF, u, v, w, tensor,
                     steps=steps, seed=seed)
