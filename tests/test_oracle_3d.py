"""Pins of the three-dimensional oracle (the scheme of Section 2 in flux form in
three directions; the paper states the model for dimension 2 or 3 and names
three-dimensional modelling as its outlook).

What fixes it independently of its formulas:
  * with one layer (nz = 1) and no couplings to z it is the 2D scheme, bit for bit;
  * an isotropic constant tensor gives the textbook 7-point Laplacian with
    mirrored (Neumann) ghost cells;
  * the exact eigenmodes cos(p pi x) cos(q pi y) cos(r pi z) of the no-flux
    Laplacian decay by the closed-form factor for a diagonal tensor, and the
    highest mode is stable exactly up to the step bound;
  * zero boundary flux conserves mass, the operator is symmetric with the
    constants as null space, and relabelling the axes relabels the result.
"""
import math

import numpy as np
import pytest

import oracle


def rng(k):
    return np.random.Generator(np.random.PCG64(3000 + k))


def spd_field(g, shape):
    """Diagonally dominant symmetric tensors (hence positive definite)."""
    axx, ayy, azz = (g.uniform(1.0, 2.0, shape) for _ in range(3))
    axy, axz, ayz = (g.uniform(-0.3, 0.3, shape) for _ in range(3))
    return [axx, ayy, azz, axy, axz, ayz]


def centres(n, l=1.0):
    return (np.arange(n) + 0.5) * (l / n)


def test_3d_one_layer_is_the_2d_scheme(orc=oracle):
    nx, ny = 13, 9
    g = rng(1)
    shape = (1, ny, nx)
    axx, ayy, axy = g.uniform(0.5, 2.0, shape), g.uniform(0.5, 2.0, shape), g.uniform(-0.4, 0.4, shape)
    A = [axx, ayy, g.uniform(0.5, 2.0, shape), axy, np.zeros(shape), np.zeros(shape)]
    u, v, w = (g.uniform(0.1, 0.9, shape) for _ in range(3))
    prm = (12.5, 1.0, 0.05, 70.0, 60.0)
    got = orc.step3(u, v, w, A, prm, 1e-5, 1.3, 0.7, 0.2)
    ref = orc.step(u[0], v[0], w[0], axx[0], axy[0], ayy[0], prm, 1e-5, 1.3, 0.7)
    assert all(np.array_equal(x[0], y) for x, y in zip(got, ref))


def test_3d_isotropic_is_7point_laplacian(orc=oracle):
    nx, ny, nz, lx, ly, lz = 6, 5, 7, 1.0, 2.0, 0.5
    g = rng(2)
    W = g.random((nz, ny, nx))
    lam = 0.7
    ones = np.ones_like(W)
    A = [lam * ones, lam * ones, lam * ones, 0 * ones, 0 * ones, 0 * ones]
    got = orc.div_w3(W, A, lx, ly, lz)
    P = np.pad(W, 1, mode="edge")      # mirrored ghost cells
    c = P[1:-1, 1:-1, 1:-1]
    idx, idy, idz = nx / lx, ny / ly, nz / lz
    ref = lam * ((P[1:-1, 1:-1, 2:] - 2 * c + P[1:-1, 1:-1, :-2]) * idx**2 +
                 (P[1:-1, 2:, 1:-1] - 2 * c + P[1:-1, :-2, 1:-1]) * idy**2 +
                 (P[2:, 1:-1, 1:-1] - 2 * c + P[:-2, 1:-1, 1:-1]) * idz**2)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def _mode(nx, ny, nz, p, q, r):
    X = centres(nx)[None, None, :]
    Y = centres(ny)[None, :, None]
    Z = centres(nz)[:, None, None]
    return np.cos(p * math.pi * X) * np.cos(q * math.pi * Y) * np.cos(r * math.pi * Z)


@pytest.mark.parametrize("p,q,r", [(1, 2, 1), (3, 0, 2)])
def test_3d_eigenmode_decay_diagonal_tensor(p, q, r, orc=oracle):
    nx, ny, nz = 10, 8, 6
    ax, ay, az = 1.3, 0.4, 0.9
    W0 = _mode(nx, ny, nz, p, q, r)
    ones = np.ones_like(W0)
    A = [ax * ones, ay * ones, az * ones, 0 * ones, 0 * ones, 0 * ones]
    mu = 4 * ax * nx**2 * math.sin(p * math.pi / (2 * nx)) ** 2 + \
        4 * ay * ny**2 * math.sin(q * math.pi / (2 * ny)) ** 2 + \
        4 * az * nz**2 * math.sin(r * math.pi / (2 * nz)) ** 2
    dt = orc.stable_dt3(A, 0.0, 0.5)
    prm = (0.0, 0.0, 0.0, 0.0, 0.0)
    n = 300
    _, _, W = orc.run3(0 * ones, 0 * ones, W0, A, prm, dt, n)
    assert np.max(np.abs(W - (1.0 - dt * mu) ** n * W0)) <= 1e-12


@pytest.mark.parametrize("s", [0.95, 1.05])
def test_3d_step_bound_is_the_stability_limit(s, orc=oracle):
    nx, ny, nz = 8, 6, 10
    W0 = _mode(nx, ny, nz, nx - 1, ny - 1, nz - 1)
    ones = np.ones_like(W0)
    lam = 0.8
    A = [lam * ones, lam * ones, lam * ones, 0 * ones, 0 * ones, 0 * ones]
    dt = orc.stable_dt3(A, 0.0, s)
    _, _, W = orc.run3(0 * ones, 0 * ones, W0, A, (0.0,) * 5, dt, 60)
    amp = np.max(np.abs(W))
    assert (amp < 0.1) if s < 1 else (amp > 3.0), amp


def test_3d_mass_conservation(orc=oracle):
    nx, ny, nz = 9, 7, 5
    g = rng(4)
    A = spd_field(g, (nz, ny, nx))
    u, v, w = (g.uniform(0.1, 0.9, (nz, ny, nx)) for _ in range(3))
    prm = (3.0, 0.0, 0.3, 0.0, 0.0)
    dt = orc.stable_dt3(A, prm[2], 0.9)
    m0 = orc.mass3(u, v, w)
    U, V, W = orc.run3(u, v, w, A, prm, dt, 200)
    m1 = orc.mass3(U, V, W)
    assert abs(m1[1] - m0[1]) <= 1e-13 * m0[1] and abs(m1[2] - m0[2]) <= 1e-13 * m0[2]


def test_3d_operator_symmetry_and_null_space(orc=oracle):
    nx, ny, nz = 6, 5, 4
    g = rng(5)
    A = spd_field(g, (nz, ny, nx))
    f, h = g.random((nz, ny, nx)), g.random((nz, ny, nx))
    lhs = np.sum(orc.div_w3(f, A) * h)
    rhs = np.sum(f * orc.div_w3(h, A))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert np.max(np.abs(orc.div_w3(np.full((nz, ny, nx), 0.37), A))) == 0.0
    U = g.uniform(0.0, 0.9, (nz, ny, nx))
    lv = np.sum(orc.div_v3(U, f) * h)
    rv = np.sum(f * orc.div_v3(U, h))
    assert abs(lv - rv) <= 1e-12 * abs(lv)


def test_3d_relabelled_axes(orc=oracle):
    nx, ny, nz = 7, 5, 4
    g = rng(6)
    A = spd_field(g, (nz, ny, nx))
    W = g.random((nz, ny, nx))
    got = orc.div_w3(W, A, 1.0, 1.5, 0.5)
    # x -> y -> z -> x: new axes (x', y', z') = (z, x, y); arrays are (z, y, x)
    perm = lambda F: np.ascontiguousarray(np.transpose(F, (1, 2, 0)))    # (y, x, z) as (z', y', x')
    axx, ayy, azz, axy, axz, ayz = A
    A2 = [perm(azz), perm(axx), perm(ayy), perm(axz), perm(ayz), perm(axy)]
    got2 = orc.div_w3(perm(W), A2, 0.5, 1.0, 1.5)
    assert np.max(np.abs(perm(got) - got2)) <= 1e-12 * np.max(np.abs(got))
    U, V = g.uniform(0.0, 0.9, (nz, ny, nx)), g.random((nz, ny, nx))
    gv = orc.div_v3(U, V, 1.0, 1.5, 0.5)
    gv2 = orc.div_v3(perm(U), perm(V), 0.5, 1.0, 1.5)
    assert np.max(np.abs(perm(gv) - gv2)) <= 1e-12 * np.max(np.abs(gv))


def test_3d_step_bound_covers_the_largest_eigenvalue(orc=oracle):
    """The bound must not exceed 1 / (2 lambda_max (idx^2 + idy^2 + idz^2)) for any
    cell, whatever its off-diagonal couplings (lambda_max from a library
    eigen-solver)."""
    nx, ny, nz, lx, ly, lz = 5, 4, 3, 1.0, 0.8, 1.2
    g = rng(7)
    shape = (nz, ny, nx)
    A = spd_field(g, shape)
    # one strongly coupled cell whose first row dominates
    A[0][1, 2, 3], A[3][1, 2, 3], A[4][1, 2, 3] = 2.5, 1.2, 1.1
    A[1][1, 2, 3], A[5][1, 2, 3], A[2][1, 2, 3] = 1.4, 0.1, 1.3
    q = (nx / lx) ** 2 + (ny / ly) ** 2 + (nz / lz) ** 2
    M = np.stack([np.stack([A[0], A[3], A[4]], -1), np.stack([A[3], A[1], A[5]], -1),
                  np.stack([A[4], A[5], A[2]], -1)], -2)
    lmax = float(np.max(np.linalg.eigvalsh(M)))
    dt = orc.stable_dt3(A, 0.01, 1.0, lx, ly, lz)
    assert dt <= 1.0 / (2.0 * lmax * q)


def test_3d_mass_closed_forms(orc=oracle):
    """Masses on a box that is neither a cube nor unit-sized, with a different
    number of cells along each axis, against the integrals they approximate.
    A constant c has mass c * lx * ly * lz; the midpoint rule is exact for
    linear fields, so x, y and z at the cell centres have masses
    lx^2/2 * ly * lz, ly^2/2 * lx * lz and lz^2/2 * lx * ly.  A cell volume
    that dropped a factor or took the wrong axis's cell count fails one of
    them."""
    nx, ny, nz, lx, ly, lz = 11, 6, 9, 1.7, 0.6, 2.3
    shape = (nz, ny, nx)
    one = np.ones(shape)
    m = orc.mass3(0.8 * one, 1.5 * one, 0.25 * one, lx, ly, lz)
    vol = lx * ly * lz
    assert np.allclose(m, [0.8 * vol, 1.5 * vol, 0.25 * vol], rtol=1e-13, atol=0.0)
    z, y, x = np.meshgrid(centres(nz, lz), centres(ny, ly), centres(nx, lx), indexing="ij")
    m = orc.mass3(x, y, z, lx, ly, lz)
    want = [lx * lx / 2 * ly * lz, ly * ly / 2 * lx * lz, lz * lz / 2 * lx * ly]
    assert np.allclose(m, want, rtol=1e-13, atol=0.0)
