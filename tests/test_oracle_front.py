"""Pins of the oracle's front diagnostics (tumour front, tissue front, interstitial
gap) and of its LeVeque-Yee front speed, and the paper's two invasion types
(Section 2) reproduced by the oracle's dynamics.

What fixes them independently of the formulas:
  * piecewise-linear ramps have their threshold crossings at known points, which
    linear interpolation between cell centres recovers exactly;
  * a profile translated by a distance changes the mass by exactly that
    distance times the jump across the front (for a smooth profile saturated at
    both ends the midpoint sum is exact to rounding), so the speed of a profile
    moved by a known amount is recovered;
  * the Gatenby-Gawlinski reactions fix the state behind the tumour front: the
    normal cells tend to 1 - d w there when d w < 1 (coexistence, heterogeneous
    invasion) and to 0 when d > 1 (homogeneous invasion), and the gap between
    the tumour and the healthy tissue opens for large d.
"""
import math

import numpy as np
import pytest

import oracle


def cell_x(nx, lx=1.0):
    return (np.arange(nx) + 0.5) * (lx / nx)


def test_front_diag_ramps_exact(orc=oracle):
    nx, ny, lx = 120, 7, 2.0
    x = cell_x(nx, lx)
    g = np.random.Generator(np.random.PCG64(41))
    av = g.uniform(0.3, 0.8, ny)            # tumour crossing per row
    au = av + g.uniform(0.1, 0.6, ny)       # tissue crossing per row
    sv = g.uniform(0.05, 0.2, ny)           # ramp widths (several cells)
    su = g.uniform(0.05, 0.2, ny)
    v = np.clip(0.5 + (av[:, None] - x[None, :]) / sv[:, None], 0.0, 1.0)
    u = np.clip(0.25 + (x[None, :] - au[:, None]) / su[:, None], 0.0, 1.0)
    f = orc.front_diag(u, v, 0.25, 0.5, lx)
    assert f["rows_front"] == ny and f["rows_gap"] == ny
    assert math.isclose(f["tumour"][0], av.mean(), rel_tol=1e-13)
    assert math.isclose(f["tumour"][1], av.min(), rel_tol=1e-13)
    assert math.isclose(f["tumour"][2], av.max(), rel_tol=1e-13)
    assert math.isclose(f["tissue"][0], au.mean(), rel_tol=1e-13)
    assert math.isclose(f["tissue"][2], au.max(), rel_tol=1e-13)
    gap = au - av
    assert math.isclose(f["gap"][0], gap.mean(), rel_tol=1e-12)
    assert math.isclose(f["gap"][1], gap.min(), rel_tol=1e-12)
    assert math.isclose(f["gap"][2], gap.max(), rel_tol=1e-12)


def test_front_diag_edge_cases(orc=oracle):
    nx, ny = 10, 4
    x = cell_x(nx)
    u = np.zeros((ny, nx))
    v = np.zeros((ny, nx))
    v[1, :] = 1.0                            # tumour everywhere: front at the last centre, no tissue ahead
    v[2, :4] = 1.0                           # step: front interpolated half way to the next centre
    u[2, 6:] = 1.0                           # tissue step two cells further
    v[3, 0] = 0.6                            # tiny tumour, tissue already at threshold next to it
    u[3, :] = 0.3
    f = orc.front_diag(u, v, 0.25, 0.5)
    assert f["rows_front"] == 3 and f["rows_gap"] == 2
    xv = [x[-1], x[3] + 0.5 / nx, x[0] + (0.6 - 0.5) / 0.6 / nx]
    assert math.isclose(f["tumour"][1], min(xv), rel_tol=1e-14)
    assert math.isclose(f["tumour"][2], max(xv), rel_tol=1e-14)
    # row 2: tissue crossing interpolated from u=0 at x[5] to u=1 at x[6]; row 3:
    # u at the tumour front's cell already above threshold, so the tissue front is
    # the next centre
    xu = [x[6] - 0.75 / nx, x[1]]
    assert math.isclose(f["tissue"][1], min(xu), rel_tol=1e-14)
    assert math.isclose(f["tissue"][2], max(xu), rel_tol=1e-14)
    empty = orc.front_diag(np.zeros((3, 5)), np.zeros((3, 5)))
    assert empty["rows_front"] == 0 and empty["rows_gap"] == 0 and empty["gap"][1] == math.inf


def test_leveque_yee_recovers_a_translation(orc=oracle):
    nx, ny, lx, ly = 800, 3, 4.0, 0.5
    x = cell_x(nx, lx)
    dx, dy = lx / nx, ly / ny
    width, behind, ahead = 0.08, 0.9, 0.1
    prof = lambda a: ahead + (behind - ahead) * 0.5 * (1.0 - np.tanh((x - a) / width))
    m0 = np.tile(prof(1.3), (ny, 1)).sum() * dx * dy
    m1 = np.tile(prof(1.3 + 0.37), (ny, 1)).sum() * dx * dy
    s = orc.front_speed(m0, m1, 2.0, 2.5, ly, behind, ahead)
    assert math.isclose(s, 0.37 / 0.5, rel_tol=1e-12)


def _invasion(d, T, nx=100, lx=1.0, orc=oracle, Delta2=0.01):
    ny, ly = 2, 2.0 * lx / nx
    x = cell_x(nx, lx)
    v0 = np.tile((x < 0.2).astype(float), (ny, 1))
    u0 = np.ones((ny, nx))
    w0 = np.zeros((ny, nx))
    ones = np.ones((ny, nx))
    prm = (d, 1.0, Delta2, 70.0, 70.0)
    dt = orc.stable_dt(ones, 0 * ones, ones, prm[2], 0.9, lx, ly)
    u, v, w, _ = orc.run(u0, v0, w0, ones, 0 * ones, ones, prm, dt, int(T / dt), lx, ly)
    return u, v, w, orc.front_diag(u, v, 0.25, 0.5, lx)


def test_heterogeneous_invasion_coexists(orc=oracle):
    d = 0.5
    u, v, w, f = _invasion(d, 8.0, orc=orc)
    # well behind the front: v near its capacity and u at the coexistence value
    ub, wb = u[0, 3], w[0, 3]
    assert v[0, 3] > 0.9 and 0.3 < ub < 0.7
    assert abs(ub - (1.0 - d * wb)) < 0.02, (ub, wb)
    assert f["gap"][2] < 2.0 / 100          # no interstitial gap


def test_homogeneous_invasion_degrades_and_opens_a_gap(orc=oracle):
    fronts = []
    for d in (0.5, 2.0, 12.5):
        u, v, w, f = _invasion(d, 3.0, orc=orc)
        fronts.append(f["tumour"][0])
        if d > 1:
            assert u[0, 5] < 0.15, (d, u[0, 5])
        if d == 12.5:
            assert f["gap"][1] > 10.0 / 100 and u[0, 5] < 1e-3
    assert fronts[0] < fronts[1] < fronts[2]   # more aggressive invasion travels faster


def test_gap_onset_bound_and_tumour_diffusivity(orc=oracle):
    """Ahead of the tumour front u' = u (1 - u - d w) >= 0 once u <= 1 - d max w,
    so while d w stays below 1 - theta_u the tissue cannot fall below theta_u
    and no gap opens.  With rho3 = delta3 the acid at the tumour front stays
    below 1/2, so d = 1.5 opens no gap even with slow tumour diffusion; d = 3
    opens one only when the tumour diffuses slowly (Delta2 = 0.001 against
    0.01), the dependence on the diffusion rates of Section 2.  Channel of
    128 cells, t = 4."""
    nx = 128
    h = 1.0 / nx
    res = {}
    for d, D2 in ((1.5, 0.001), (3.0, 0.001), (3.0, 0.01)):
        u, v, w, f = _invasion(d, 4.0, nx=nx, orc=orc, Delta2=D2)
        last = int(np.nonzero(v[0] >= 0.5)[0].max())
        res[(d, D2)] = (f["gap"][0], 0.5 * (w[0, last] + w[0, last + 1]))
    gap, wf = res[(1.5, 0.001)]
    assert wf < 0.5 and 1.5 * wf < 1.0 - 0.25 and gap < h, res
    assert res[(3.0, 0.01)][0] < h, res
    assert res[(3.0, 0.001)][0] > 1.5 * h, res
