"""Writes ansatz_param_shift.json: oracle parameter-shift gradients of the
32-qubit, 8-layer Ry/Rz + CNOT-ladder ansatz (512 angles uniform in
[0, 2 pi), seed 1004), loss sum_i <Z_i Z_{i+1}>, at chi_max = 256.

At chi_max = 256 the circuit is not truncated (a ladder of 8 layers keeps
every bond at rank <= 2^8; the oracle's summed discarded weight is rounding,
about 1e-14), so the two-term shift rule for R_P(t) = exp(-i t P/2) is exact
(Mitarai et al., PRA 98, 032309 (2018)).  Only the oracle and the seeded
input generators are called.  16 angles, drawn with seed 4040, are
evaluated (two oracle forwards each).

Run from the repository root:  python tests/golden/make_ansatz_param_shift.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2601_04422_amd import workloads as W  # noqa: E402

N, NL, CHI, COUNT, PICK_SEED = 32, 8, 256, 16, 4040


def main():
    O.set_threads(len(os.sched_getaffinity(0)))
    angles = W.ansatz_angles(N, NL)
    paulis = W.zz_chain(N)
    coeffs = [1.0] * len(paulis)
    make = lambda a: W.ansatz_gates(a, N, NL)  # noqa: E731
    idx = sorted(int(p) for p in np.random.default_rng(PICK_SEED).choice(angles.size, COUNT,
                                                                          replace=False))
    t0 = time.perf_counter()
    base = O.run_gates(N, CHI, 0.0, make(angles))
    loss = O.loss_pauli_sum(base, paulis, coeffs)
    g = O.parameter_shift(make, angles, N, CHI, 0.0, paulis, coeffs, which=idx)
    out = {"n": N, "layers": NL, "chi_max": CHI, "cutoff": 0.0, "angle_seed": 1004,
           "pick_seed": PICK_SEED, "loss": loss, "sum_eps": base.stats()["sum_eps"],
           "indices": idx, "grad": [float(g[p]) for p in idx],
           "source": "oracle forward passes, two-term parameter shift"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ansatz_param_shift.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} in {time.perf_counter() - t0:.0f} s")


if __name__ == "__main__":
    main()
