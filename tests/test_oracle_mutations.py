"""The oracle's pins catch plausible mistakes (CPU only).

Each case copies oracle/fem_oracle.c, plants one mistake (a dropped term, a wrong sign,
a transposed index, a missing factor), compiles the copy, routes the oracle through it and
runs the pins that should notice: at least one must fail.  The mistakes live only in the
temporary copy.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_action as pins
import test_oracle_curved as curved
import test_oracle_min_det as mindet

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "fem_oracle.c")

MUTATIONS = {
    "nh_drop_log_term": ("S[i][j] = mu * (F[i][j] - FiT) + lam * lnJ * FiT;",
                         "S[i][j] = mu * (F[i][j] - FiT);",
                         [lambda: pins.test_hyper_residual_is_energy_gradient(pins.F_NH, 2, 2),
                          lambda: pins.test_hyper_vjp_at_zero_is_elasticity(pins.F_NH, 2, 2)]),
    "nh_sign_of_cofactor": ("S[i][j] = mu * (F[i][j] - FiT) + lam * lnJ * FiT;",
                            "S[i][j] = mu * (F[i][j] + FiT) + lam * lnJ * FiT;",
                            [lambda: pins.test_hyper_invariances(pins.F_NH, 2, 2)]),
    "jacobian_transposed": ("J[i][r] += x[g][i] * gdq[g * d + r];",
                            "J[i][r] += x[g][r] * gdq[g * d + i];",
                            [lambda: pins.test_elasticity_equals_exact_assembly(2, 2, 2, pins.LAME)]),
    "no_abs_det": ("double detJ = fabs(geometry(d, ng, x, gdphi + (int64_t)q * ng * d, J, K));\n            const double W = w[q] * detJ;\n            if (form == OR_MASS",
                   "double detJ = geometry(d, ng, x, gdphi + (int64_t)q * ng * d, J, K);\n            const double W = w[q] * detJ;\n            if (form == OR_MASS",
                   [lambda: pins.test_mass_partition_of_unity(3, 2)]),
    "curved_geometry_frozen_at_first_point": (
        "double detJ = fabs(geometry(d, ng, x, gdphi + (int64_t)q * ng * d, J, K));\n            const double W = w[q] * detJ;\n            if (form == OR_MASS",
        "double detJ = fabs(geometry(d, ng, x, gdphi, J, K));\n            const double W = w[q] * detJ;\n            if (form == OR_MASS",
        [lambda: curved.test_curved_mass_moments(2, 4),
         lambda: curved.test_curved_laplace_patch_test(2, 2)]),
    "weight_without_det": ("const double W = w[q] * detJ;\n            if (form == OR_MASS || form == OR_HELMHOLTZ)",
                           "const double W = w[q];\n            if (form == OR_MASS || form == OR_HELMHOLTZ)",
                           [lambda: pins.test_mass_partition_of_unity(2, 2)]),
    "elasticity_half_shear": ("S[i][j] = 2.0 * mu * eps + (i == j ? lam * tr : 0.0);",
                              "S[i][j] = mu * eps + (i == j ? lam * tr : 0.0);",
                              [lambda: pins.test_elasticity_equals_exact_assembly(2, 2, 2, pins.LAME)]),
    "contraction_transposed": ("out[a * d + c] += dq[a * d + r] * E[c][r];\n            }\n        }\n        for (int a = 0; a < nloc; ++a)\n            for (int c = 0; c < ncomp; ++c)",
                               "out[a * d + c] += dq[a * d + r] * E[r][c];\n            }\n        }\n        for (int a = 0; a < nloc; ++a)\n            for (int c = 0; c < ncomp; ++c)",
                               [lambda: pins.test_elasticity_equals_exact_assembly(2, 2, 2, pins.LAME)]),
    "vjp_tangent_index": ("+ (mu - lam * lnJ) * Fi[j][k] * Fi[l][i]",
                          "+ (mu - lam * lnJ) * Fi[k][j] * Fi[l][i]",
                          [lambda: pins.test_hyper_vjp_against_finite_differences(pins.F_NH, 2, 2, 2)]),
    "energy_sign": ("return 0.5 * mu * (trC - d) - mu * lnJ + 0.5 * lam * lnJ * lnJ;",
                    "return 0.5 * mu * (trC - d) + mu * lnJ + 0.5 * lam * lnJ * lnJ;",
                    [lambda: pins.test_hyper_residual_is_energy_gradient(pins.F_NH, 2, 2)]),
    "mass_test_function_dropped": ("out[a] += phi[q * nloc + a] * e;",
                                   "out[a] += e / nloc;",
                                   [lambda: pins.test_mass_equals_exact_assembly(2, 2, 2)]),
    "svk_stress_transposed_product": ("S[i][j] += F[i][k] * S2[k][j];",
                                      "S[i][j] += S2[i][k] * F[k][j];",
                                      [lambda: pins.test_hyper_invariances(pins.F_SVK, 2, 2),
                                       lambda: pins.test_svk_homogeneous_one_cell("shear")]),
    "svk_energy_missing_half": ("return 0.5 * lam * trE * trE + mu * EE;",
                                "return lam * trE * trE + mu * EE;",
                                [lambda: pins.test_hyper_residual_is_energy_gradient(pins.F_SVK, 2, 2)]),
    "svk_tangent_drops_geometric_term": ("C = (i == k ? S2[l][j] : 0.0) + lam * F[i][j] * F[k][l]",
                                         "C = lam * F[i][j] * F[k][l]",
                                         [lambda: pins.test_hyper_vjp_against_finite_differences(pins.F_SVK, 2, 2, 2)]),
    "laplace_gradient_not_mapped": ("                            gu[j] += uloc[a] * dq[a * d + r] * K[r][j];",
                                    "                            gu[j] += uloc[a] * dq[a * d + r] * K[j][r];",
                                    [lambda: pins.test_laplace_helmholtz_equal_exact_assembly(2, 2, 2)]),
    "helmholtz_mass_term_dropped": ("if (form == OR_MASS || form == OR_HELMHOLTZ) {\n                double uq",
                                    "if (form == OR_MASS) {\n                double uq",
                                    [lambda: pins.test_laplace_helmholtz_equal_exact_assembly(2, 2, 2)]),
    "min_det_f_keeps_first_point": ("            if (det < mn)\n                mn = det;",
                                    "            if (q == 0 && cell == 0)\n                mn = det;",
                                    [lambda: mindet.test_quadratic_displacement_extreme_point(2, 2, 0, 0.3, "conical")]),
    "min_det_f_without_identity": ("F[i][j] = (i == j ? 1.0 : 0.0) + G[i][j];\n            double det = inverse(d, F, Fi);",
                                   "F[i][j] = G[i][j];\n            double det = inverse(d, F, Fi);",
                                   [lambda: mindet.test_zero_displacement_gives_one(2, 1, "conical")]),
    "colouring_ignores_conflicts": ("if ((masks[nd * nwords + c / 64] >> (c % 64)) & 1u) {",
                                    "if (0) {",
                                    [lambda: pins.test_colouring_valid_and_greedy(2, 6, 1)]),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new, checks = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mut = tmp_path / "fem_oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", str(so), str(mut), "-lm"],
                   check=True)
    caught = 0
    with oracle.using_library(str(so)):
        for check in checks:
            try:
                with np.errstate(all="ignore"):
                    check()
            except AssertionError:
                caught += 1
    assert caught >= 1, f"no pin noticed the planted mistake {name}"
