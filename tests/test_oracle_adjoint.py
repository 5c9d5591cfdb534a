"""Pins of the oracle's discrete adjoint against the (already pinned) forward step.

One step F of eq. (3) is a polynomial of degree two in the state (u^2, u w, and the
mobility times a difference in the tumour flux) and affine in each reaction
parameter and in the tensor (a, b, c).  A central difference of a quadratic or
affine map is exact up to rounding, so the dot-product identities
<(F(x+e d) - F(x-e d)) / 2e, lam> = <d, (dF/dx)^T lam> hold to rounding level and
pin the adjoint term by term.  Over many steps the map is no longer quadratic;
there the reverse sweep is checked against central differences of the loss.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2006_01748_amd import workloads as wl

SEED = wl.BASE_SEED + 900
PRM = (12.5, 1.3, 0.07, 60.0, 45.0)


def rng(k):
    return np.random.Generator(np.random.PCG64(SEED + k))


def setup(nx=13, ny=9, k=0):
    g = rng(k)
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    lam = tuple(g.standard_normal((ny, nx)) for _ in range(3))
    dt = oracle.stable_dt(a, b, c, PRM[2], 0.8, 1.0, 0.7)
    return g, (u, v, w), (a, b, c), lam, dt


def dot3(x, y):
    return sum(float(np.sum(p * q)) for p, q in zip(x, y))


@pytest.mark.parametrize("nx,ny", [(13, 9), (1, 6), (7, 1), (2, 3)])
def test_state_adjoint_dot_identity(nx, ny):
    g, x, abc, lam, dt = setup(nx, ny, 1)
    d = tuple(g.standard_normal((ny, nx)) for _ in range(3))
    eps = 1e-3
    fp = oracle.step(*(xi + eps * di for xi, di in zip(x, d)), *abc, PRM, dt, 1.0, 0.7)
    fm = oracle.step(*(xi - eps * di for xi, di in zip(x, d)), *abc, PRM, dt, 1.0, 0.7)
    jd = tuple((p - m) / (2 * eps) for p, m in zip(fp, fm))
    lam0, _, _ = oracle.adjoint_step(*x, *abc, PRM, dt, lam, 1.0, 0.7)
    lhs, rhs = dot3(jd, lam), dot3(d, lam0)
    scale = math.sqrt(dot3(jd, jd) * dot3(lam, lam))
    assert abs(lhs - rhs) <= 1e-11 * scale, (lhs, rhs)


def test_parameter_gradients_exact_differences():
    g, x, abc, lam, dt = setup(11, 14, 2)
    _, _, gp = oracle.adjoint_step(*x, *abc, PRM, dt, lam, 1.0, 0.7)
    for k in range(5):
        e = 1e-3 * max(1.0, abs(PRM[k]))
        p1 = list(PRM)
        p2 = list(PRM)
        p1[k] += e
        p2[k] -= e
        fp = oracle.step(*x, *abc, p1, dt, 1.0, 0.7)
        fm = oracle.step(*x, *abc, p2, dt, 1.0, 0.7)
        fd = dot3(tuple((p - m) / (2 * e) for p, m in zip(fp, fm)), lam)
        assert abs(fd - gp[k]) <= 1e-9 * max(abs(fd), 1e-12) + 1e-13, (k, fd, gp[k])


def test_tensor_gradients_exact_differences():
    g, x, abc, lam, dt = setup(12, 10, 3)
    _, gabc, _ = oracle.adjoint_step(*x, *abc, PRM, dt, lam, 1.0, 0.7)
    for _ in range(3):
        d = tuple(g.standard_normal(abc[0].shape) for _ in range(3))
        eps = 1e-4
        fp = oracle.step(*x, *(t + eps * di for t, di in zip(abc, d)), PRM, dt, 1.0, 0.7)
        fm = oracle.step(*x, *(t - eps * di for t, di in zip(abc, d)), PRM, dt, 1.0, 0.7)
        fd = dot3(tuple((p - m) / (2 * eps) for p, m in zip(fp, fm)), lam)
        an = dot3(gabc, d)
        assert abs(fd - an) <= 1e-9 * abs(an), (fd, an)
    # each of a, b, c separately (a wrong component would cancel in a sum)
    for comp in range(3):
        d = [np.zeros_like(abc[0]) for _ in range(3)]
        d[comp] = g.standard_normal(abc[0].shape)
        eps = 1e-4
        fp = oracle.step(*x, *(t + eps * di for t, di in zip(abc, d)), PRM, dt, 1.0, 0.7)
        fm = oracle.step(*x, *(t - eps * di for t, di in zip(abc, d)), PRM, dt, 1.0, 0.7)
        fd = dot3(tuple((p - m) / (2 * eps) for p, m in zip(fp, fm)), lam)
        an = float(np.sum(gabc[comp] * d[comp]))
        assert abs(fd - an) <= 1e-9 * abs(an), (comp, fd, an)


def test_eig_chain_rule():
    g = rng(4)
    l1, l2, th = wl.random_eig(g, 8, 6)
    ga, gb, gc = (g.standard_normal(l1.shape) for _ in range(3))
    g1, g2, gt = oracle.eig_backward(l1, l2, th, ga, gb, gc)
    for comp, gref in enumerate((g1, g2, gt)):
        d = [np.zeros_like(l1) for _ in range(3)]
        d[comp] = g.standard_normal(l1.shape)
        eps = 1e-6
        ap = oracle.tensor_from_eig(*(x + eps * di for x, di in zip((l1, l2, th), d)))
        am = oracle.tensor_from_eig(*(x - eps * di for x, di in zip((l1, l2, th), d)))
        fd = dot3(tuple((p - m) / (2 * eps) for p, m in zip(ap, am)), (ga, gb, gc))
        an = float(np.sum(gref * d[comp]))
        assert abs(fd - an) <= 1e-8 * abs(an), (comp, fd, an)


def _loss_and_lam(x_final, target, dxdy):
    v, w = x_final[1], x_final[2]
    L = 0.5 * dxdy * (np.sum((v - target[0]) ** 2) + np.sum((w - target[1]) ** 2))
    lam = (np.zeros_like(v), dxdy * (v - target[0]), dxdy * (w - target[1]))
    return L, lam


def test_reverse_sweep_against_loss_differences():
    nx, ny, N = 16, 12, 40
    g, x0, abc, _, dt = setup(nx, ny, 5)
    dt = oracle.stable_dt(*abc, PRM[2], 0.8)
    dxdy = 1.0 / (nx * ny)
    target = (g.uniform(0, 1, (ny, nx)), g.uniform(0, 1, (ny, nx)))

    def loss(x, abc_, prm):
        xf = oracle.run(*x, *abc_, prm, dt, N)[:3]
        return _loss_and_lam(xf, target, dxdy)[0]

    xf = oracle.run(*x0, *abc, PRM, dt, N)[:3]
    L0, lamN = _loss_and_lam(xf, target, dxdy)
    lam0, gabc, gp = oracle.adjoint_run(*x0, *abc, PRM, dt, N, lamN)
    # state direction
    d = tuple(g.standard_normal((ny, nx)) for _ in range(3))
    eps = 1e-5
    fd = (loss(tuple(a + eps * b for a, b in zip(x0, d)), abc, PRM) -
          loss(tuple(a - eps * b for a, b in zip(x0, d)), abc, PRM)) / (2 * eps)
    assert abs(fd - dot3(lam0, d)) <= 1e-6 * abs(fd)
    # tensor direction
    d = tuple(0.1 * g.standard_normal((ny, nx)) for _ in range(3))
    fd = (loss(x0, tuple(a + eps * b for a, b in zip(abc, d)), PRM) -
          loss(x0, tuple(a - eps * b for a, b in zip(abc, d)), PRM)) / (2 * eps)
    assert abs(fd - dot3(gabc, d)) <= 1e-6 * abs(fd)
    # each scalar parameter
    for k in range(5):
        e = 1e-5 * max(1.0, abs(PRM[k]))
        p1, p2 = list(PRM), list(PRM)
        p1[k] += e
        p2[k] -= e
        fd = (loss(x0, abc, p1) - loss(x0, abc, p2)) / (2 * e)
        assert abs(fd - gp[k]) <= 1e-6 * abs(fd) + 1e-14, (k, fd, gp[k])
