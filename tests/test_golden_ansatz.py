"""The stored parameter-shift gradients of the 32-qubit ansatz
(tests/golden/ansatz_param_shift.json, written by make_ansatz_param_shift.py
from oracle forwards only) are reproduced by the oracle: the loss and one
stored entry, recomputed here (no GPU)."""
import json
import os

import numpy as np

from oracle import oracle as O
from paper_2601_04422_amd import workloads as W


def test_stored_parameter_shift_reproduces():
    path = os.path.join(os.path.dirname(__file__), "golden", "ansatz_param_shift.json")
    ref = json.load(open(path))
    n, nl, chi = ref["n"], ref["layers"], ref["chi_max"]
    O.set_threads(min(8, len(os.sched_getaffinity(0))))
    angles = W.ansatz_angles(n, nl, ref["angle_seed"])
    paulis = W.zz_chain(n)
    coeffs = [1.0] * len(paulis)
    make = lambda a: W.ansatz_gates(a, n, nl)  # noqa: E731
    base = O.run_gates(n, chi, 0.0, make(angles))
    assert base.stats()["sum_eps"] < 1e-12  # untruncated: the shift rule is exact
    assert abs(O.loss_pauli_sum(base, paulis, coeffs) - ref["loss"]) < 1e-12
    p = ref["indices"][-1]
    g = O.parameter_shift(make, angles, n, chi, 0.0, paulis, coeffs, which=[p])
    assert abs(g[p] - ref["grad"][-1]) < 1e-12
    assert np.isfinite(ref["grad"]).all() and len(ref["grad"]) == len(ref["indices"]) == 16
