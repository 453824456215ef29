"""Plant plausible mistakes in copies of the oracle and check that the pins
catch each one (a pin suite that a dropped term, a wrong sign, a lost
conjugate or a transposed operand survives would not pin anything).

The copies are compiled from the oracle source with one text substitution
each; the real oracle is untouched.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import oracle as O

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "tnsim_oracle.c")

MUTANTS = {
    "lambda weight dropped": ("double w = lr ? lr[c] : 1.0;", "double w = 1.0;"),
    "conjugate dropped in right site": ("cplx w = conj(U[(size_t)j * rows + r]) / N;",
                                        "cplx w = U[(size_t)j * rows + r] / N;"),
    "gate transposed": ("acc += G[(2 * sp + tp) * 4 + j] * v[j];",
                        "acc += G[j * 4 + (2 * sp + tp)] * v[j];"),
    "rotation sign": ("x[i] = c * xv - s * yt;", "x[i] = c * xv + s * yt;"),
    "cutoff equality kept": ("if (tail[k] <= cutoff * W) { kc = k; break; }",
                             "if (tail[k] < cutoff * W) { kc = k; break; }"),
    "swap orientation": ("= G[(2 * tp + sp) * 4 + 2 * t + s];", "= G[(2 * sp + tp) * 4 + 2 * s + t];"),
    "1q gate transposed": ("A[(a * 2 + 0) * b_n + b] = U[0] * x0 + U[1] * x1;",
                           "A[(a * 2 + 0) * b_n + b] = U[0] * x0 + U[2] * x1;"),
    "no renormalisation": ("for (int j = 0; j < k; j++) nl[j] = sig[j] / N;",
                           "for (int j = 0; j < k; j++) nl[j] = sig[j];"),
    "bra not conjugated": ("cplx w = conj(B[((size_t)a * 2 + s) * ra + b]);",
                           "cplx w = B[((size_t)a * 2 + s) * ra + b];"),
    "descending sort reversed": ("if (sa > sb) return -1;\n  if (sa < sb) return 1;",
                                 "if (sa < sb) return -1;\n  if (sa > sb) return 1;"),
    "householder reflector factor": ("cplx f = 2.0 * d / vnorm2;", "cplx f = d / vnorm2;"),
    "M^H not conjugated": ("Y[(size_t)i * cols + j] = conj(M[(size_t)j * rows + i]);",
                           "Y[(size_t)i * cols + j] = M[(size_t)j * rows + i];"),
    "swap chain not undone": ("for (int j = a + 1; j < b; j++) {", "for (int j = b; j < b; j++) {"),
    "far qubit orientation lost": (
        "q0 == a ? apply_2q_adjacent(m, a, a + 1, G) : apply_2q_adjacent(m, a + 1, a, G);",
        "apply_2q_adjacent(m, a, a + 1, G);"),
    "sampling ignores the environment": ("for (int ap = 0; ap < la; ap++) t += E[(size_t)a * la + ap] * w[ap];",
                                         "for (int ap = 0; ap < la; ap++) t += (a == ap) * w[ap];"),
    "sampling threshold on the other bit": ("u[(size_t)shot * n + q] < p0 / (p0 + p1) ? 0 : 1",
                                            "u[(size_t)shot * n + q] < p1 / (p0 + p1) ? 0 : 1"),
    "sampling projects the other outcome": ("const cplx *wb = bit ? w1 : w0;",
                                            "const cplx *wb = bit ? w0 : w1;"),
    "canonical sweep without the Schmidt weight": (
        "m->A[b + 1][((size_t)a * 2 + t) * chiR + c] * (lr ? lr[c] : 1.0);",
        "m->A[b + 1][((size_t)a * 2 + t) * chiR + c] * 1.0;"),
    "canonical sweep drops the remainder": (
        "for (int e = 0; e < w; e++) nB[(size_t)j * w + e] += f * m->A[q + 1][(size_t)c * w + e];",
        "for (int e = 0; e < w; e++) nB[(size_t)j * w + e] += (j == c) * m->A[q + 1][(size_t)c * w + e];"),
    "propagation: right factor without conjugate": (
        "for (int i = 0; i < 4; i++) acc += conj(Ug[r * 4 + i]) * Gm[e * 4 + i];",
        "for (int i = 0; i < 4; i++) acc += Ug[r * 4 + i] * Gm[e * 4 + i];"),
    "propagation: gate orientation ignored": (
        "const int row = q0 == a ? 2 * xp + yp : 2 * yp + xp;",
        "const int row = 2 * xp + yp;"),
    "propagation: propagating index order mixed up": (
        "const int li = q == a ? l : r * L + l, ri = q == b ? c : r * R + c;",
        "const int li = q == a ? l : r * L + l, ri = q == b ? c : c * rg + r;"),
    "canonical sweep rotates with conj(U)": (
        "for (int j = 0; j < k; j++) nA[(size_t)i * k + j] += f * U[(size_t)j * rows + a];",
        "for (int j = 0; j < k; j++) nA[(size_t)i * k + j] += f * conj(U[(size_t)j * rows + a]);"),
}

PIN_CALLS = [
    pins.test_product_state_closed_forms,
    pins.test_small_brickwork_matches_statevector,
    lambda: pins.test_random_circuits_with_1q_and_reversed_gates(11),
    pins.test_ghz_golden,
    pins.test_lambda_are_schmidt_values_and_norm,
    pins.test_truncation_error_equals_discarded_weight,
    lambda: pins.test_jacobi_svd_against_numpy((8, 16)),
    lambda: pins.test_jacobi_svd_against_numpy((64, 64)),
    pins.test_truncation_rule,
    pins.test_layer_order_independence,
    pins.test_nonlocal_gates_match_statevector,
    pins.test_nonlocal_ghz_closed_form,
    pins.test_sampling_matches_brute_force,
    pins.test_sampling_in_any_gauge,
    pins.test_sampling_product_state_closed_form,
    pins.test_sampling_ghz_closed_form,
    pins.test_canonicalize_generic_gauge_against_brute_force,
    pins.test_canonicalize_leaves_a_canonical_state_unchanged,
    pins.test_canonicalize_truncation_is_the_optimal_cut,
    lambda: pins.test_propagation_matches_statevector("haar"),
    pins.test_propagation_ghz_and_operator_rank,
    pins.test_propagation_truncation_is_a_right_to_left_schmidt_cut,
]


def _build_mutant(old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = os.path.join(tmp, "mut.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(tmp, "libmut.so")
    subprocess.check_call(["gcc", "-O1", "-fcx-fortran-rules", "-fPIC", "-shared", "-std=gnu99",
                           "-o", so, path, "-lm"])
    return so


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name):
    old, new = MUTANTS[name]
    with tempfile.TemporaryDirectory() as tmp:
        so = _build_mutant(old, new, tmp)
        O.use_library(so)
        caught = []
        try:
            for call in PIN_CALLS:
                try:
                    call()
                except (AssertionError, O.OracleError, ValueError, np.linalg.LinAlgError):
                    caught.append(getattr(call, "__name__", "lambda"))
        finally:
            O.use_library(None)
    assert caught, f"planted mistake '{name}' survived every pin"
