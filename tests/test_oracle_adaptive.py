"""Pins of the oracle's adaptive step size (Section 2: a new step size after
every iteration, chosen for stability of the explicit scheme).

The rule itself is a reading (the paper prints none): the largest dt whose
per-cell Gershgorin number equals the safety factor.  What pins it is what the
mathematics fixes independently of that formula:
  * for an isotropic constant tensor it is the textbook bound of the explicit
    five-point heat equation, dt = s / (2 D (1/dx^2 + 1/dy^2)), with D the
    larger of the two diffusivities;
  * on the exact highest eigenmode of the no-flux Laplacian (the DCT-II mode
    cos((n-1) pi x)), the explicit scheme at that step decays for s < 1 and
    grows for s > 1, by the closed-form factor 1 - dt D mu per step; with the
    normal cells at a constant density u0 the tumour-cell diffusivity is
    Delta2 (1 - u0), so the threshold pins the mobility factor too.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2006_01748_amd import workloads as wl


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_adaptive_isotropic_is_textbook_bound(orc=oracle):
    nx, ny, lx, ly = 12, 20, 1.5, 0.8
    idx2, idy2 = (nx / lx) ** 2, (ny / ly) ** 2
    ones = np.ones((ny, nx))
    zeros = np.zeros((ny, nx))
    for lam, D2 in ((3.0, 0.5), (0.2, 1.7)):
        dt = orc.adaptive_dt(zeros, lam * ones, zeros, lam * ones, D2, 0.9, lx, ly)
        ref = 0.9 / (2.0 * max(lam, D2) * (idx2 + idy2))
        assert math.isclose(dt, ref, rel_tol=4e-16), (lam, D2, dt, ref)
    # a constant rotated tensor: the Gershgorin number of the nine-point stencil
    # (diagonal 2(a idx^2 + c idy^2), off-diagonal sum |b| idx idy)
    lam1, lam2, th = np.full((ny, nx), 2.0), np.full((ny, nx), 0.5), np.full((ny, nx), 0.7)
    a, b, c = orc.tensor_from_eig(lam1, lam2, th)
    dt = orc.adaptive_dt(ones, a, b, c, 0.01, 0.5, lx, ly)
    g = 2 * (a[0, 0] * idx2 + c[0, 0] * idy2) + abs(b[0, 0]) * math.sqrt(idx2 * idy2)
    assert math.isclose(dt, 0.5 / g, rel_tol=1e-14)


def _highest_mode(nx, ny):
    X, Y = wl.cell_centres(nx, ny)
    return np.cos((nx - 1) * math.pi * X) * np.cos((ny - 1) * math.pi * Y)


@pytest.mark.parametrize("u0", [0.0, 0.75])
@pytest.mark.parametrize("s", [0.95, 1.05])
def test_adaptive_stability_threshold_on_highest_mode(u0, s, orc=oracle):
    nx, ny = 14, 10
    idx, idy = nx, ny
    D2 = 0.8
    V0 = 0.5 + 0.25 * _highest_mode(nx, ny)
    ones = np.ones((ny, nx))
    lam = 1e-3                           # acid diffusion far below the tumour cells'
    # delta1 = 1 and w = 1 - u0 hold u at u0 exactly: u(1 - u - delta1 w) = 0
    prm = (1.0, 0.0, D2, 0.0, 0.0)
    u = np.full((ny, nx), u0)
    w = np.full((ny, nx), 1.0 - u0)
    n = 40
    U, V, W, log, t = orc.run_adaptive(u, V0, w, lam * ones, 0 * ones, lam * ones, prm, s, n)
    assert np.array_equal(U, u) and np.array_equal(W, w)
    D = D2 * (1.0 - u0)
    mu = 4 * idx**2 * math.sin((nx - 1) * math.pi / (2 * nx)) ** 2 + \
        4 * idy**2 * math.sin((ny - 1) * math.pi / (2 * ny)) ** 2
    dt = log[0]
    assert np.all(log == dt)
    g = 1.0 - dt * D * mu
    ref = 0.5 + 0.25 * g**n * _highest_mode(nx, ny)
    assert np.max(np.abs(V - ref)) <= 1e-12
    amp = np.max(np.abs(V - 0.5)) / 0.25
    if s < 1:
        assert abs(g) < 1 and amp < 0.1, (g, amp)
    else:
        assert abs(g) > 1 and amp > 2.0, (g, amp)
    assert math.isclose(t, n * dt, rel_tol=1e-15)


def test_adaptive_follows_the_state(orc=oracle):
    """Each step's size is the rule applied to the state that step starts from,
    and the time is the running sum of the steps."""
    nx, ny = 17, 13
    g = rng(21)
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    prm = (12.5, 1.0, 0.3, 70.0, 60.0)
    U, V, W, log, t = orc.run_adaptive(u, v, w, a, b, c, prm, 0.9, 6, t0=0.25)
    x = (u, v, w)
    tt = 0.25
    for k in range(6):
        dt = orc.adaptive_dt(x[0], a, b, c, prm[2], 0.9)
        assert dt == log[k]
        assert math.isclose(orc.diagnostics(*x, a, b, c, prm[2], dt)["cfl"], 0.9, rel_tol=2e-16)
        x = orc.step(*x, a, b, c, prm, dt)
        tt += dt
    assert all(np.array_equal(p, q) for p, q in zip(x, (U, V, W)))
    assert t == tt
    # zero steps: nothing changes
    U0, V0, W0, log0, t0 = orc.run_adaptive(u, v, w, a, b, c, prm, 0.9, 0, t0=1.0)
    assert np.array_equal(U0, u) and t0 == 1.0 and log0.size == 0
