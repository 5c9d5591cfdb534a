"""Pins of the FP64 oracle against facts fixed outside it.

Each test ties the oracle to something it does not compute itself: the stencil
coefficients printed in Tables 1 and 2 (stored as golden data), textbook
operators, closed-form discrete eigenmodes, closed-form ODE solutions,
conservation and symmetry identities, polynomial exactness and the convergence
order of a manufactured solution.  Grids are rectangular (nx != ny) wherever the
x/y roles could be confused.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2006_01748_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SEED = wl.BASE_SEED + 77


def rng(k=0):
    return np.random.Generator(np.random.PCG64(SEED + k))


def _load_table(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _apply_table(table, fields, scales, nx, ny):
    """Evaluate a transcribed stencil on interior cells 1..n-2."""
    main = fields[table["field"]]
    out = np.zeros((ny - 2, nx - 2))
    J, I = np.mgrid[1:ny - 1, 1:nx - 1]
    for e in table["entries"]:
        di, dj = e["offset"]
        coef = np.zeros_like(out)
        for (k, name, (oi, oj), sc) in e["terms"]:
            fac = 1.0 if name == "1" else fields[name][J + oj, I + oi]
            coef = coef + k * fac * scales[sc]
        out += coef * main[J + dj, I + di]
    return out


# ---------------------------------------------------------------------------
# P1: flux form against the printed stencils (Tables 1 and 2)

@pytest.mark.parametrize("nx,ny,lx,ly", [(17, 11, 1.0, 1.0), (24, 31, 1.3, 0.7)])
def test_p1_table2_transcription(orc, nx, ny, lx, ly):
    g = rng(1)
    a, b, c = wl.random_abc(g, nx, ny)
    W = g.uniform(-1, 1, (ny, nx))
    idx, idy = nx / lx, ny / ly
    sc = {"idx2": idx * idx, "idy2": idy * idy, "idxy": idx * idy}
    ref = _apply_table(_load_table("table2_stencil.json"), {"W": W, "a": a, "b": b, "c": c},
                       sc, nx, ny)
    got = orc.div_w(W, a, b, c, lx, ly)[1:-1, 1:-1]
    scale = np.abs(W).max() * max(sc.values()) * 4.0
    assert np.max(np.abs(got - ref)) <= 1e-13 * scale


@pytest.mark.parametrize("nx,ny,lx,ly", [(17, 11, 1.0, 1.0), (24, 31, 1.3, 0.7)])
def test_p1_table1_transcription(orc, nx, ny, lx, ly):
    g = rng(2)
    U = g.uniform(0, 1, (ny, nx))
    V = g.uniform(-1, 1, (ny, nx))
    idx, idy = nx / lx, ny / ly
    sc = {"idx2": idx * idx, "idy2": idy * idy}
    ref = _apply_table(_load_table("table1_stencil.json"), {"V": V, "U": U}, sc, nx, ny)
    got = orc.div_v(U, V, lx, ly)[1:-1, 1:-1]
    scale = np.abs(V).max() * max(sc.values()) * 4.0
    assert np.max(np.abs(got - ref)) <= 1e-13 * scale


# ---------------------------------------------------------------------------
# P2: special cases that reduce to the textbook Neumann five-point Laplacian

def neumann_laplacian(nx, ny, lx, ly):
    def lap1(n, h):
        main = -2.0 * np.ones(n)
        main[0] = main[-1] = -1.0
        if n == 1:
            main[0] = 0.0
        return sp.diags([np.ones(n - 1), main, np.ones(n - 1)], [-1, 0, 1]) / (h * h)
    return (sp.kron(sp.identity(ny), lap1(nx, lx / nx)) + sp.kron(lap1(ny, ly / ny), sp.identity(nx))).tocsr()


@pytest.mark.parametrize("nx,ny", [(13, 9), (1, 7), (6, 1), (2, 2)])
def test_p2_isotropic_is_textbook_laplacian(orc, nx, ny):
    g = rng(3)
    W = g.uniform(-1, 1, (ny, nx))
    D = 1.7
    a = np.full((ny, nx), D)
    c = a.copy()
    b = np.zeros((ny, nx))
    L = neumann_laplacian(nx, ny, 1.0, 1.3)
    ref = D * (L @ W.ravel()).reshape(ny, nx)
    got = orc.div_w(W, a, b, c, 1.0, 1.3)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-12 * np.abs(ref).max() + 1e-300)


def test_p2_mobility_special_cases(orc):
    nx, ny = 12, 8
    g = rng(4)
    V = g.uniform(-1, 1, (ny, nx))
    L = neumann_laplacian(nx, ny, 1.0, 1.0)
    ref = (L @ V.ravel()).reshape(ny, nx)
    got0 = orc.div_v(np.zeros((ny, nx)), V)
    assert np.allclose(got0, ref, rtol=1e-13, atol=1e-12 * np.abs(ref).max())
    got1 = orc.div_v(np.ones((ny, nx)), V)
    assert np.all(got1 == 0.0)            # degenerate: no flux where U = 1


# ---------------------------------------------------------------------------
# P3: closed-form discrete eigenmodes of the Neumann operator

@pytest.mark.parametrize("p,q", [(1, 0), (2, 3), (0, 1)])
def test_p3_eigenmode_decay_w(orc, p, q):
    nx, ny, lx, ly = 20, 14, 1.0, 1.0
    X, Y = wl.cell_centres(nx, ny, lx, ly)
    W0 = np.cos(p * math.pi * X) * np.cos(q * math.pi * Y)
    A, C = 1.6, 0.45                      # a != c pins the x/y orientation
    a = np.full((ny, nx), A)
    c = np.full((ny, nx), C)
    b = np.zeros((ny, nx))
    idx, idy = nx / lx, ny / ly
    mu = A * 4 * idx**2 * math.sin(p * math.pi / (2 * nx)) ** 2 + \
         C * 4 * idy**2 * math.sin(q * math.pi / (2 * ny)) ** 2
    dt = 0.3 / (4 * max(A, C) * (idx**2 + idy**2))
    prm = (0.0, 0.0, 0.0, 0.0, 0.0)
    u0 = np.ones((ny, nx))
    v0 = np.zeros((ny, nx))
    n = 1000
    u, v, w, _ = orc.run(u0, v0, W0, a, b, c, prm, dt, n)
    ref = (1.0 - dt * mu) ** n * W0
    assert np.max(np.abs(w - ref)) <= 1e-12 * max(np.abs(W0).max() * abs(1.0 - dt * mu) ** n, 1e-300)
    assert np.all(u == 1.0) and np.all(v == 0.0)


@pytest.mark.parametrize("p,q", [(1, 1), (3, 0)])
def test_p3_eigenmode_decay_v(orc, p, q):
    nx, ny = 16, 22
    X, Y = wl.cell_centres(nx, ny)
    V0 = np.cos(p * math.pi * X) * np.cos(q * math.pi * Y)
    D2 = 0.37
    idx, idy = nx, ny
    mu = 4 * idx**2 * math.sin(p * math.pi / (2 * nx)) ** 2 + 4 * idy**2 * math.sin(q * math.pi / (2 * ny)) ** 2
    dt = 0.3 / (4 * D2 * (idx**2 + idy**2))
    prm = (0.0, 0.0, D2, 0.0, 0.0)
    ones = np.ones((ny, nx))
    u, v, w, _ = orc.run(np.zeros((ny, nx)), V0, np.zeros((ny, nx)), ones, 0 * ones, ones,
                         prm, dt, 800)
    ref = (1.0 - dt * D2 * mu) ** 800 * V0
    assert np.max(np.abs(v - ref)) <= 1e-12 * np.abs(V0).max()


# ---------------------------------------------------------------------------
# P4: conservation with zero boundary flux; P5: operator symmetry

def test_p4_mass_conservation(orc):
    nx, ny = 24, 18
    g = rng(5)
    a, b, c = wl.random_abc(g, nx, ny)
    u, v, w = wl.random_state(g, nx, ny)
    prm = (3.0, 0.0, 0.05, 0.0, 0.0)      # rho2 = rho3 = delta3 = 0
    dt = orc.stable_dt(a, b, c, prm[2], 0.9)
    m0 = orc.diagnostics(u, v, w, a, b, c, prm[2], dt)["mass"]
    u1, v1, w1, log = orc.run(u, v, w, a, b, c, prm, dt, 4000, mass_every=1000)
    for row in log:
        assert abs(row[1] - m0[1]) <= 1e-13 * abs(m0[1])
        assert abs(row[2] - m0[2]) <= 1e-13 * abs(m0[2])
    assert abs(log[-1][0] - m0[0]) > 1e-6   # u is not conserved (reactions on)


def test_p5_operator_symmetry_and_nullspace(orc):
    nx, ny = 15, 12
    g = rng(6)
    a, b, c = wl.random_abc(g, nx, ny)
    U = g.uniform(0, 1, (ny, nx))
    x = g.standard_normal((ny, nx))
    y = g.standard_normal((ny, nx))
    for L in (lambda z: orc.div_w(z, a, b, c, 1.0, 0.8), lambda z: orc.div_v(U, z, 1.0, 0.8)):
        lhs = np.sum(L(x) * y)
        rhs = np.sum(x * L(y))
        scale = np.linalg.norm(L(x)) * np.linalg.norm(y)
        assert abs(lhs - rhs) <= 1e-13 * scale
        assert abs(np.sum(L(x))) <= 1e-12 * np.linalg.norm(L(x))     # 1^T L = 0
        assert np.max(np.abs(L(np.full((ny, nx), 0.7)))) == 0.0        # L 1 = 0


# ---------------------------------------------------------------------------
# P6: homogeneous equilibria are preserved bit for bit

@pytest.mark.parametrize("state", ["normal", "tumour"])
def test_p6_equilibria_bitwise(orc, state):
    nx, ny = 19, 13
    g = rng(7)
    a, b, c = wl.random_abc(g, nx, ny)
    prm = (12.5, 1.0, 0.01, 70.0, 70.0)
    if state == "normal":
        u0, v0, w0 = np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx))
    else:
        u0, v0, w0 = np.zeros((ny, nx)), np.ones((ny, nx)), np.ones((ny, nx))
    dt = orc.stable_dt(a, b, c, prm[2], 0.9)
    u, v, w, _ = orc.run(u0, v0, w0, a, b, c, prm, dt, 10000)
    assert np.array_equal(u, u0) and np.array_equal(v, v0) and np.array_equal(w, w0)


# ---------------------------------------------------------------------------
# P7: dihedral equivariance on square grids

def test_p7_transpose_and_reflection(orc):
    n = 14
    g = rng(8)
    a, b, c = wl.random_abc(g, n, n)
    u, v, w = wl.random_state(g, n, n)
    prm = (12.5, 1.0, 0.01, 70.0, 70.0)
    dt = 1e-5
    ref = orc.step(u, v, w, a, b, c, prm, dt)
    # transpose: x <-> y, a <-> c, b unchanged
    t = orc.step(u.T, v.T, w.T, c.T, b.T, a.T, prm, dt)
    for r, s in zip(ref, t):
        assert np.array_equal(r.T, s)
    # reflection x -> 1 - x: b -> -b
    f = orc.step(u[:, ::-1], v[:, ::-1], w[:, ::-1], a[:, ::-1], -b[:, ::-1], c[:, ::-1], prm, dt)
    for r, s in zip(ref, f):
        assert np.array_equal(r[:, ::-1], s)
    # quarter turn: (i, j) -> (j, n-1-i) composes both
    rot = lambda z: np.rot90(z)
    q = orc.step(rot(u), rot(v), rot(w), rot(c), -rot(b), rot(a), prm, dt)
    for r, s in zip(ref, q):
        assert np.array_equal(rot(r), s)


# ---------------------------------------------------------------------------
# P8: reactions against closed-form ODE solutions (uniform states)

def _uniform_run(orc, u0, v0, w0, prm, T, n):
    nx, ny = 5, 4
    g = rng(9)
    a, b, c = wl.random_abc(g, nx, ny)
    st = [np.full((ny, nx), x) for x in (u0, v0, w0)]
    u, v, w, _ = orc.run(*st, a, b, c, prm, T / n, n)
    assert np.all(u == u[0, 0]) and np.all(v == v[0, 0]) and np.all(w == w[0, 0])
    return u[0, 0], v[0, 0], w[0, 0]


def test_p8_reactions_first_order_convergence(orc):
    T = 0.5
    d1, r2, r3, d3 = 0.8, 1.7, 3.0, 2.0
    u0, v0, w0 = 0.3, 0.2, 0.4
    # u: dU/dt = U (1 - d1 W0 - U) with W held fixed (rho3 = delta3 = 0)
    rr = 1.0 - d1 * w0
    U_ex = rr * u0 * math.exp(rr * T) / (rr + u0 * (math.exp(rr * T) - 1.0))
    # v: logistic with rate rho2
    V_ex = v0 * math.exp(r2 * T) / (1.0 - v0 + v0 * math.exp(r2 * T))
    # w: dW/dt = rho3 V0 - delta3 W with V held fixed (rho2 = 0)
    W_ex = r3 * v0 / d3 + (w0 - r3 * v0 / d3) * math.exp(-d3 * T)
    errs = []
    for n in (200, 400, 800):
        u, _, _ = _uniform_run(orc, u0, v0, w0, (d1, 0.0, 0.0, 0.0, 0.0), T, n)
        _, v, _ = _uniform_run(orc, u0, v0, w0, (0.0, r2, 0.0, 0.0, 0.0), T, n)
        _, _, w = _uniform_run(orc, u0, v0, w0, (0.0, 0.0, 0.0, r3, d3), T, n)
        errs.append((abs(u - U_ex), abs(v - V_ex), abs(w - W_ex)))
    for k in range(3):
        for lvl in range(2):
            ratio = errs[lvl][k] / errs[lvl + 1][k]
            assert 1.85 < ratio < 2.15, (k, errs)
        assert errs[-1][k] < 2e-3


# ---------------------------------------------------------------------------
# P9: manufactured solution, second order in h with dt ~ h^2

def _mms_functions():
    sym = pytest.importorskip("sympy")
    t, x, y = sym.symbols("t x y")
    pi = sym.pi
    U = sym.Rational(1, 2) + sym.Rational(1, 4) * sym.cos(pi * x) * sym.cos(pi * y) * sym.exp(-t)
    V = sym.Rational(2, 5) + sym.Rational(1, 5) * sym.cos(pi * x) * sym.cos(2 * pi * y) * (1 + t)
    W = sym.Rational(3, 10) + sym.Rational(1, 10) * sym.cos(2 * pi * x) * sym.cos(pi * y) * sym.exp(t)
    a = sym.Rational(3, 2) + sym.Rational(1, 2) * sym.cos(pi * x) * sym.cos(pi * y)
    c = sym.Rational(6, 5) + sym.Rational(3, 10) * sym.sin(2 * pi * x) * sym.cos(pi * y)
    b = sym.Rational(2, 5) * sym.sin(pi * x) * sym.sin(pi * y)     # zero on the boundary
    d1, r2, D2, r3, d3 = 1.0, 1.0, 0.5, 1.0, 1.5
    div = lambda fx, fy: sym.diff(fx, x) + sym.diff(fy, y)
    SU = sym.diff(U, t) - (U * (1 - U) - d1 * U * W)
    SV = sym.diff(V, t) - (r2 * V * (1 - V) + D2 * div((1 - U) * sym.diff(V, x), (1 - U) * sym.diff(V, y)))
    SW = sym.diff(W, t) - (r3 * V - d3 * W + div(a * sym.diff(W, x) + b * sym.diff(W, y),
                                                  b * sym.diff(W, x) + c * sym.diff(W, y)))
    f = lambda e: sym.lambdify((t, x, y), e, "numpy")
    return dict(U=f(U), V=f(V), W=f(W), a=f(a), b=f(b), c=f(c), SU=f(SU), SV=f(SV), SW=f(SW),
                prm=(d1, r2, D2, r3, d3))


def test_p9_manufactured_solution_second_order(orc):
    F = _mms_functions()
    T = 0.02
    errs = []
    for n in (16, 32, 64):
        X, Y = wl.cell_centres(n, n)
        full = lambda f, tt: np.broadcast_to(f(tt, X, Y), X.shape).astype(np.float64)
        a, b, c = full(F["a"], 0.0), full(F["b"], 0.0), full(F["c"], 0.0)
        nsteps = int(round(T * n * n / 0.05))          # dt = 0.05 h^2
        dt = T / nsteps
        u, v, w = full(F["U"], 0.0), full(F["V"], 0.0), full(F["W"], 0.0)
        for k in range(nsteps):
            tk = k * dt
            src = (full(F["SU"], tk), full(F["SV"], tk), full(F["SW"], tk))
            u, v, w = orc.step(u, v, w, a, b, c, F["prm"], dt, sources=src)
        e = max(np.abs(u - full(F["U"], T)).max(), np.abs(v - full(F["V"], T)).max(),
                np.abs(w - full(F["W"], T)).max())
        errs.append(e)
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(1.85 <= o <= 2.15 for o in orders), (errs, orders)


# ---------------------------------------------------------------------------
# P10: polynomial exactness; P11: linearity

def test_p10_polynomials(orc):
    nx, ny, lx, ly = 21, 16, 1.0, 0.9
    X, Y = wl.cell_centres(nx, ny, lx, ly)
    A, B, C = 1.3, -0.45, 0.8
    a, b, c = (np.full((ny, nx), z) for z in (A, B, C))
    inner = (slice(2, -2), slice(2, -2))
    for W, expect in ((X * X, 2 * A), (Y * Y, 2 * C), (X * Y, 2 * B)):
        got = orc.div_w(W, a, b, c, lx, ly)[inner]
        assert np.allclose(got, expect, rtol=0, atol=1e-9)


def test_p11_linearity(orc):
    nx, ny = 11, 14
    g = rng(10)
    a1, b1, c1 = wl.random_abc(g, nx, ny)
    a2, b2, c2 = wl.random_abc(g, nx, ny)
    W1, W2 = g.standard_normal((ny, nx)), g.standard_normal((ny, nx))
    s, t = 0.7, -1.9
    L = lambda W, a, b, c: orc.div_w(W, a, b, c)
    lhs = L(s * W1 + t * W2, a1, b1, c1)
    rhs = s * L(W1, a1, b1, c1) + t * L(W2, a1, b1, c1)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())
    lhs = L(W1, a1 + a2, b1 + b2, c1 + c2)
    rhs = L(W1, a1, b1, c1) + L(W1, a2, b2, c2)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())


# ---------------------------------------------------------------------------
# tensor map, step bound, diagnostics

def test_tensor_from_eig_matches_eigh(orc):
    g = rng(11)
    lam1, lam2, theta = wl.random_eig(g, 9, 7)
    a, b, c = orc.tensor_from_eig(lam1, lam2, theta)
    M = np.stack([np.stack([a, b], -1), np.stack([b, c], -1)], -2)
    ev, evec = np.linalg.eigh(M)
    assert np.allclose(ev[..., 1], lam1, rtol=1e-14)
    assert np.allclose(ev[..., 0], lam2, rtol=1e-13)
    d = np.stack([np.cos(theta), np.sin(theta)], -1)          # principal direction
    assert np.allclose(np.abs(np.sum(evec[..., :, 1] * d, -1)), 1.0, atol=1e-12)
    lm = np.array([[orc.lambda_max(a[j, i], b[j, i], c[j, i]) for i in range(9)] for j in range(7)])
    assert np.allclose(lm, lam1, rtol=1e-14)
    assert orc.count_not_spd(a, b, c) == 0
    assert orc.count_not_spd(a, 2 * np.sqrt(a * c) + 0 * b, c) == a.size


def test_stable_dt_closed_form(orc):
    w = wl.cfg0(steps=1)
    a, b, c = w.abc
    assert orc.stable_dt(a, b, c, w.params[2], 0.2) == w.dt_closed_form
    # anisotropic constant tensor: bound follows the largest eigenvalue
    nx, ny = 10, 30
    lam1, lam2, th = np.full((ny, nx), 2.5), np.full((ny, nx), 0.5), np.full((ny, nx), 0.3)
    a, b, c = orc.tensor_from_eig(lam1, lam2, th)
    dt = orc.stable_dt(a, b, c, 0.01, 0.9)
    assert math.isclose(dt, 0.9 / (2 * 2.5 * (nx**2 + ny**2)), rel_tol=1e-14)


def test_diagnostics_closed_forms(orc):
    nx, ny, lx, ly = 8, 6, 2.0, 0.5
    u = np.full((ny, nx), 0.25)
    v = np.full((ny, nx), 0.5)
    w = np.full((ny, nx), 2.0)
    ones = np.ones((ny, nx))
    d = orc.diagnostics(u, v, w, ones, 0 * ones, ones, 0.01, 0.0, lx, ly)
    assert np.allclose(d["mass"], [0.25 * lx * ly, 0.5 * lx * ly, 2.0 * lx * ly], rtol=1e-15)
    assert d["nonfinite"] == 0
    # isotropic constant tensor at the bound's step: cfl equals the safety factor
    dt = orc.stable_dt(ones, 0 * ones, ones, 0.01, 0.6, lx, ly)
    d = orc.diagnostics(u, v, w, ones, 0 * ones, ones, 0.01, dt, lx, ly)
    assert math.isclose(d["cfl"], 0.6, rel_tol=1e-14)
    w2 = w.copy()
    w2[1, 2] = np.nan
    w2[3, 3] = np.inf
    d = orc.diagnostics(u, v, w2, ones, 0 * ones, ones, 0.01, dt, lx, ly)
    assert d["nonfinite"] == 2 and d["vmax"][2] == 2.0
