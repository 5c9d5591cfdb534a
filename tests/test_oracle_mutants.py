"""Planted mistakes in the oracle must be caught by its pins.

Each case copies the oracle's C source, applies one plausible slip (a dropped
term, a flipped sign, a swapped index or operand, a wrong coefficient), builds the
copy with gcc into a temporary directory, binds it in place of the real oracle
and runs the pin tests against it.  The case passes only if at least one pin
fails.  Everything runs on the CPU.
"""
import os
import subprocess
import tempfile

import pytest

import oracle
import test_oracle_3d as o3
import test_oracle_adaptive as adapt
import test_oracle_front as front
import test_oracle_adjoint as adj
import test_oracle_pins as pins

# (name, original text, replacement, expected number of occurrences)
MUTANTS = [
    ("cross-term sign", "+ 0.5 * (b[l] * tyl + b[r] * tyr)", "- 0.5 * (b[l] * tyl + b[r] * tyr)", 1),
    ("cross operands swapped", "b[l] * tyl + b[r] * tyr", "b[l] * tyr + b[r] * tyl", 1),
    ("cross factor 1/2 dropped", "+ 0.5 * (b[l] * txl + b[r] * txr)", "+ (b[l] * txl + b[r] * txr)", 1),
    ("a used on y faces", "0.5 * (c[l] + c[r]) * ((W[r] - W[l]) * idy)", "0.5 * (a[l] + a[r]) * ((W[r] - W[l]) * idy)", 1),
    ("idy on x faces", "0.5 * (a[l] + a[r]) * ((W[r] - W[l]) * idx)", "0.5 * (a[l] + a[r]) * ((W[r] - W[l]) * idy)", 1),
    ("tangential difference one-sided", "(W[IX(i, clampi(j + 1, ny))] - W[IX(i, clampi(j - 1, ny))])",
     "(W[IX(i, clampi(j + 1, ny))] - W[IX(i, clampi(j, ny))])", 1),
    ("hy in tx", "tx_at(nx, ny, W, i, j, hx)", "tx_at(nx, ny, W, i, j, hy)", 1),
    ("mobility of one cell", "(1.0 - 0.5 * (U[l] + U[r])) * ((V[r] - V[l]) * idx)",
     "(1.0 - U[l]) * ((V[r] - V[l]) * idx)", 1),
    ("divergence sign", "out[IX(i, j)] = (fe - fw) * idx", "out[IX(i, j)] = (fw - fe) * idx", 1),
    ("kill term without U", "(d1 * U) * W", "d1 * W", 1),
    ("Delta2 dropped", "D2 * dV[k]", "dV[k]", 1),
    ("acid rates swapped", "(r3 * V - d3 * W)", "(d3 * V - r3 * W)", 1),
    ("logistic of wrong field", "U * (1.0 - U)", "U * (1.0 - V)", 1),
    ("boundary face carries flux", "for (int i = 0; i + 1 < nx; ++i) {\n            size_t l = IX(i, j), r = IX(i + 1, j);\n            double tyl",
     "for (int i = 0; i + 1 < nx; ++i) {\n            size_t l = IX(i, j), r = IX(i + 1, j);\n            if (i == 0) FX[(size_t)j * (nx + 1)] = 0.5 * b[l] * ty_at(nx, ny, W, 0, j, hy);\n            double tyl", 1),
    ("lambda_max sign", "return m + sqrt(d * d + b * b);", "return m - sqrt(d * d + b * b);", 1),
    ("tensor map b sign", "b[k] = (lam1[k] - lam2[k]) * (sn * cs);", "b[k] = (lam2[k] - lam1[k]) * (sn * cs);", 1),
    ("adaptive dt without the mobility", "double cv = 2.0 * Delta2 * fabs(1.0 - u[k]) * (idx * idx + idy * idy);",
     "double cv = 2.0 * Delta2 * (idx * idx + idy * idy);", 1),
    ("adaptive dt from the diagonal only", "+ fabs(b[k]) * (idx * idy);", ";", 1),
    ("adaptive dt factor 2 dropped", "double cw = 2.0 * (a[k]", "double cw = (a[k]", 1),
    ("tumour front interpolated the wrong way", "xv = xv + (a - theta_v) / (a - b) * dx;",
     "xv = xv - (a - theta_v) / (a - b) * dx;", 1),
    ("first instead of last tumour cell", "if (v[IX(i, j)] >= theta_v) iv = i;",
     "if (v[IX(i, j)] >= theta_v && iv < 0) iv = i;", 1),
    ("tissue front not interpolated", "if (d < theta_u) xu = xu - (c - theta_u) / (c - d) * dx;", "", 1),
    ("front speed without the jump", "((t1 - t0) * ly * (behind - ahead))", "((t1 - t0) * ly)", 1),
]

PIN_TESTS = [
    lambda o: pins.test_p1_table2_transcription(o, 17, 11, 1.0, 1.0),
    lambda o: pins.test_p1_table1_transcription(o, 24, 31, 1.3, 0.7),
    lambda o: pins.test_p2_isotropic_is_textbook_laplacian(o, 13, 9),
    lambda o: pins.test_p2_mobility_special_cases(o),
    lambda o: pins.test_p3_eigenmode_decay_w(o, 2, 3),
    lambda o: pins.test_p3_eigenmode_decay_v(o, 1, 1),
    lambda o: pins.test_p4_mass_conservation(o),
    lambda o: pins.test_p5_operator_symmetry_and_nullspace(o),
    lambda o: pins.test_p7_transpose_and_reflection(o),
    lambda o: pins.test_p8_reactions_first_order_convergence(o),
    lambda o: pins.test_p10_polynomials(o),
    lambda o: pins.test_tensor_from_eig_matches_eigh(o),
    lambda o: pins.test_stable_dt_closed_form(o),
    lambda o: adapt.test_adaptive_isotropic_is_textbook_bound(o),
    lambda o: adapt.test_adaptive_stability_threshold_on_highest_mode(0.75, 1.05, o),
    lambda o: adapt.test_adaptive_stability_threshold_on_highest_mode(0.0, 1.05, o),
    lambda o: front.test_front_diag_ramps_exact(o),
    lambda o: front.test_front_diag_edge_cases(o),
    lambda o: front.test_leveque_yee_recovers_a_translation(o),
]


ADJ_MUTANTS = [
    ("mobility derivative sign", "lu[l] += sv * (-0.5 * (v[r] - v[l]) * idx);", "lu[l] += sv * (0.5 * (v[r] - v[l]) * idx);", 1),
    ("mirror term of ty dropped", "lw[IX(i, jm)] -= s * 0.5 * b[l] * hy;", "", 1),
    ("b gradient with the neighbour's ty", "gb[l] += s * 0.5 * tyl;", "gb[l] += s * 0.5 * tyr;", 1),
    ("kill-term adjoint uses w", "- dt * d1 * u[k] * lu1[k]", "- dt * d1 * w[k] * lu1[k]", 1),
    ("Delta2 gradient without divV", "gp[2] += dt * dV[k] * lv1[k];", "gp[2] += dt * lv1[k];", 1),
    ("theta chain rule sign", "(-ga[k] * s2 + gc[k] * s2 + gb[k] * c2)", "(ga[k] * s2 - gc[k] * s2 + gb[k] * c2)", 1),
    ("c gradient scaled by idx", "gc[l] += s * 0.5 * (w[r] - w[l]) * idy;", "gc[l] += s * 0.5 * (w[r] - w[l]) * idx;", 1),
    ("growth adjoint of v", "(1.0 + dt * r2 * (1.0 - 2.0 * v[k]))", "(1.0 + dt * r2 * (1.0 - v[k]))", 1),
]

MUTANTS_3D = [
    ("3D tz one-sided", "return (W[IX3(i, j, clamp3(k + 1, nz))] - W[IX3(i, j, clamp3(k - 1, nz))]) * hz;",
     "return (W[IX3(i, j, clamp3(k + 1, nz))] - W[IX3(i, j, k)]) * hz;", 1),
    ("3D axz on the y faces", "0.5 * (axy[l] * txl + axy[r] * txr) + 0.5 * (ayz[l] * tzl + ayz[r] * tzr);",
     "0.5 * (axy[l] * txl + axy[r] * txr) + 0.5 * (axz[l] * tzl + axz[r] * tzr);", 1),
    ("3D z face without its cross terms", "0.5 * (axz[l] * txl + axz[r] * txr) + 0.5 * (ayz[l] * tyl + ayz[r] * tyr);",
     "0.0;", 1),
    ("3D z mobility of one cell", "GZ[l] = (1.0 - 0.5 * (U[l] + U[r])) * ((V[r] - V[l]) * idz);",
     "GZ[l] = (1.0 - U[l]) * ((V[r] - V[l]) * idz);", 1),
    ("3D idz on the z divergence dropped", "+ (FZ[c] - fb) * idz;", "+ (FZ[c] - fb);", 1),
    ("3D bound without the off-diagonals", "double r0 = fabs(axx[c]) + fabs(axy[c]) + fabs(axz[c]);",
     "double r0 = fabs(axx[c]);", 1),
    ("3D mass without the z cell height", "double vol = (lx / nx) * (ly / ny) * (lz / nz);",
     "double vol = (lx / nx) * (ly / ny);", 1),
    ("3D mass with the x cell count on z", "double vol = (lx / nx) * (ly / ny) * (lz / nz);",
     "double vol = (lx / nx) * (ly / ny) * (lz / nx);", 1),
]

PINS_3D = [
    lambda o: o3.test_3d_one_layer_is_the_2d_scheme(o),
    lambda o: o3.test_3d_isotropic_is_7point_laplacian(o),
    lambda o: o3.test_3d_eigenmode_decay_diagonal_tensor(1, 2, 1, o),
    lambda o: o3.test_3d_step_bound_is_the_stability_limit(1.05, o),
    lambda o: o3.test_3d_mass_conservation(o),
    lambda o: o3.test_3d_operator_symmetry_and_null_space(o),
    lambda o: o3.test_3d_relabelled_axes(o),
    lambda o: o3.test_3d_step_bound_covers_the_largest_eigenvalue(o),
    lambda o: o3.test_3d_mass_closed_forms(o),
]

ADJ_PINS = [
    lambda: adj.test_state_adjoint_dot_identity(13, 9),
    lambda: adj.test_state_adjoint_dot_identity(1, 6),
    lambda: adj.test_parameter_gradients_exact_differences(),
    lambda: adj.test_tensor_gradients_exact_differences(),
    lambda: adj.test_eig_chain_rule(),
]


def _build_mutant(tmp, src_text, target="ggfv_oracle.c"):
    srcs = []
    for path in oracle.sources():
        text = open(path).read()
        if os.path.basename(path) == target:
            text = src_text
        dst = os.path.join(tmp, os.path.basename(path))
        with open(dst, "w") as f:
            f.write(text)
        srcs.append(dst)
    lib = os.path.join(tmp, "libmutant.so")
    subprocess.run(["gcc", *oracle.CFLAGS, *srcs, "-o", lib, "-lm"], check=True)
    return lib


@pytest.mark.parametrize("name,old,new,count", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, count):
    base = open(oracle._SRC).read()
    assert base.count(old) == count, f"mutation anchor for '{name}' not found"
    mutated = base.replace(old, new)
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(tmp, mutated)
        oracle.build(force=False)
        prev = oracle.use_library(lib)
        caught = []
        try:
            for k, pin in enumerate(PIN_TESTS):
                try:
                    pin(oracle)
                except AssertionError:
                    caught.append(k)
                    break
        finally:
            oracle.restore_library(prev)
    assert caught, f"no pin caught the planted mistake '{name}'"


@pytest.mark.parametrize("name,old,new,count", ADJ_MUTANTS, ids=[m[0] for m in ADJ_MUTANTS])
def test_adjoint_pins_catch_mutant(name, old, new, count):
    base = open(oracle._SRC_ADJ).read()
    assert base.count(old) == count, f"mutation anchor for '{name}' not found"
    mutated = base.replace(old, new)
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(tmp, mutated, "ggfv_oracle_adjoint.c")
        oracle.build(force=False)
        prev = oracle.use_library(lib)
        caught = False
        try:
            for pin in ADJ_PINS:
                try:
                    pin()
                except AssertionError:
                    caught = True
                    break
        finally:
            oracle.restore_library(prev)
    assert caught, f"no adjoint pin caught the planted mistake '{name}'"


@pytest.mark.parametrize("name,old,new,count", MUTANTS_3D, ids=[m[0] for m in MUTANTS_3D])
def test_3d_pins_catch_mutant(name, old, new, count):
    base = open(oracle._SRC_3D).read()
    assert base.count(old) == count, f"mutation anchor for '{name}' not found"
    mutated = base.replace(old, new)
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(tmp, mutated, "ggfv_oracle3d.c")
        oracle.build(force=False)
        prev = oracle.use_library(lib)
        caught = False
        try:
            for pin in PINS_3D:
                try:
                    pin(oracle)
                except AssertionError:
                    caught = True
                    break
        finally:
            oracle.restore_library(prev)
    assert caught, f"no 3D pin caught the planted mistake '{name}'"
