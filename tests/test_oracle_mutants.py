"""Plant plausible mistakes in a copy of the oracle and check the pins see them.

Each mutant is a one-token edit of ``oracle/nurbs_oracle.c`` (a dropped term,
a flipped sign, a closed interval, a missing weight), compiled on the CPU
into a private shared library.  The pin suite of ``test_oracle_pins`` must
fail on every mutant; this is what makes the oracle trustworthy as the
reference for the HIP path.
"""
import os
import subprocess

import pytest

from oracle import oracle as O
from tests import test_oracle_curve_pins as TC
from tests import test_oracle_loss_pins as TL
from tests import test_oracle_scattered_pins as TS
from tests import test_oracle_pins as T

MUTANTS = {
    # half-open degree-0 indicator read as closed
    "closed_indicator": ("(U[i] <= u && u < U[i + 1]) ? 1.0 : 0.0",
                         "(U[i] <= u && u <= U[i + 1]) ? 1.0 : 0.0"),
    # beta term of the Cox-de Boor recursion dropped (dense)
    "drop_beta": ("                v += b * Ni1;\n                vdu += b * du[i + 1] - Ni1 / den2;",
                  "                v += 0.0 * Ni1;\n                vdu += b * du[i + 1] - Ni1 / den2;"),
    # wrong sign of dalpha/dU_{i+d} (dense)
    "alpha_knot_sign": ("g[i + d] += -Ni * (u - U[i]) / (den1 * den1);",
                        "g[i + d] += Ni * (u - U[i]) / (den1 * den1);"),
    # beta partial w.r.t. U_{i+1} uses the wrong numerator (dense)
    "beta_knot_index": ("g[i + 1] += Ni1 * (U[i + d + 1] - u) / (den2 * den2);",
                        "g[i + 1] += Ni1 * (U[i + d] - u) / (den2 * den2);"),
    # rational basis without its weight
    "dP_no_weight": ("const double R = Ni * Nj * w[ij] / Wsum;",
                     "const double R = Ni * Nj / Wsum;"),
    # sign error in the weight derivative
    "dW_sign": ("(Ni * Nj * Pij[x] * Wsum - NR[x] * Ni * Nj) / W2",
                "(Ni * Nj * Pij[x] * Wsum + NR[x] * Ni * Nj) / W2"),
    # transposed weight index in the forward sum
    "w_transposed": ("const double wij = w[(size_t)i * nv_c + j];",
                     "const double wij = w[(size_t)j * nu_c + i];"),
    # dS/dN_i drops the denominator's derivative term
    "dSdN_drop": ("for (int x = 0; x < 3; ++x) c += g[x] * (num[x] / Wsum - NR[x] / W2 * den);\n                rowsum[ci] = c;",
                  "for (int x = 0; x < 3; ++x) c += g[x] * (num[x] / Wsum);\n                rowsum[ci] = c;"),
    # last-span rule lost: u == U_{n+1} falls off the end
    # curve: sign error in (P_i - C) of the weight and knot derivatives
    "curve_dW_sign": ("pg += (P[(size_t)i * dim + x] - C[x]) * g[x];",
                      "pg += (P[(size_t)i * dim + x] + C[x]) * g[x];"),
    # curve: rational basis without its weight
    "curve_dP_no_weight": ("dP[(size_t)i * dim + x] += N[i] * w[i] / Wsum * g[x];",
                           "dP[(size_t)i * dim + x] += N[i] / Wsum * g[x];"),
    # curve: dC/du drops the denominator's derivative
    "curve_du_drop": ("(Au[x] * Wsum - A[x] * Wu) / (Wsum * Wsum)",
                      "(Au[x] * Wsum) / (Wsum * Wsum)"),
    # loss: squared distance used where the norm belongs
    "loss_squared": ("    const double d = sqrt(s);\n", "    const double d = s;\n"),
    # loss: the second (target-to-point) Chamfer term dropped
    "loss_one_sided": ("        cd += pair_dist(dim, P + (size_t)i * dim, Q + (size_t)j * dim, dir);",
                       "        cd += 0.0 * pair_dist(dim, P + (size_t)i * dim, Q + (size_t)j * dim, dir);"),
    # loss: last index wins ties of the nearest-point decision
    "loss_tie_last": ("            if (d < bd) { bd = d; best = j; }", "            if (d <= bd) { bd = d; best = j; }"),
    # loss: gradient of the second term sent to the target's index
    "loss_grad_index": ("            for (int x = 0; x < dim; ++x) gcd[(size_t)i * dim + x] += dir[x];\n        if (db[j]",
                        "            for (int x = 0; x < dim; ++x) gcd[(size_t)(j % n) * dim + x] += dir[x];\n        if (db[j]"),
    # scattered: per-pair gradients overwrite instead of accumulating
    "scattered_overwrite": ("for (size_t i = 0; rc == OR_OK && i < 3 * ncp; ++i) dP[i] += tP[i];",
                            "for (size_t i = 0; rc == OR_OK && i < 3 * ncp; ++i) dP[i] = tP[i];"),
    # scattered: v read from the wrong slot of the pair
    "scattered_v_slot": ("uv + 2 * (size_t)k, uv + 2 * (size_t)k + 1,\n                             S + 3",
                         "uv + 2 * (size_t)k, uv + 2 * (size_t)k,\n                             S + 3"),
    "no_last_span": ("    if (u >= U[n + 1]) {\n        val[n] = 1.0;\n    } else {",
                     "    if (0) {\n        val[n] = 1.0;\n    } else {"),
}

PINS = [
    (T.test_span_matches_bisect_random, ()),
    (T.test_partition_of_unity_nonneg_local_support, ()),
    (T.test_bernstein_closed_form, (3,)),
    (T.test_uniform_quadratic_and_cubic_pieces, ()),
    (T.test_basis_knot_derivative_finite_difference_and_sum_rule, ()),
    (T.test_dense_equals_local_basis, ()),
    (T.test_forward_matches_de_boor, (0,)),
    (T.test_forward_matches_de_boor, (1,)),
    (T.test_quarter_circle_cylinder, ()),
    (T.test_endpoint_interpolation, ()),
    (T.test_grad_ctrl_and_weights_fd, (False,)),
    (T.test_grad_invariants_translation_and_weight_scale, ()),
    (T.test_grad_knots_fd, (False,)),
    (T.test_grad_knots_shift_and_scale_invariance, ()),
    (T.test_dense_equals_local_surface, ()),
    (TC.test_quarter_circle, ()),
    (TC.test_rational_bezier_closed_form, (3,)),
    (TC.test_curve_is_surface_edge, (0,)),
    (TC.test_finite_differences, ()),
    (TC.test_invariants, ()),
    (TL.test_nearest_exact_on_integer_lattice_first_index_wins, ()),
    (TL.test_identity_and_symmetry, ()),
    (TL.test_shifted_copy_closed_form, (3,)),
    (TL.test_hand_worked_example, ()),
    (TL.test_finite_differences, (3,)),
    (TS.test_shuffled_grid_equals_grid, (3, 3)),
    (TS.test_scattered_finite_differences, ()),
]


@pytest.fixture
def mutant_lib(tmp_path):
    saved = (O._lib, O.LIB, O.SRC)

    def make(name):
        old, new = MUTANTS[name]
        text = open(saved[2]).read()
        assert text.count(old) == 1, f"mutation anchor for {name} not unique"
        src = tmp_path / f"{name}.c"
        src.write_text(text.replace(old, new))
        so = tmp_path / f"lib_{name}.so"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-o", str(so), str(src), "-lm"])
        O._lib, O.LIB, O.SRC = None, str(so), str(src)
        os.utime(so)
    yield make
    O._lib, O.LIB, O.SRC = saved


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(mutant_lib, name):
    mutant_lib(name)
    caught = []
    for fn, args in PINS:
        try:
            fn(*args)
        except (AssertionError, O.OracleError, ValueError, FloatingPointError):
            caught.append(fn.__name__)
    assert caught, f"no pin caught mutant {name}"
