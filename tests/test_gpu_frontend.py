"""Circuits read from OpenQASM and fused (host front end), run on the GPU,
against the oracle running the same circuit unfused."""
import cmath
import math

import numpy as np
import pytest

from gpu_helpers import mps_fidelity_gpu_vs_oracle
from oracle import oracle as O
from paper_2601_04422_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2601_04422_amd import tnsim

    return tnsim


def _qft_program(n, x):
    lines = ['OPENQASM 2.0;', 'include "qelib1.inc";', f"qreg q[{n}];"]
    lines += [f"x q[{q}];" for q in range(n) if (x >> (n - 1 - q)) & 1]
    for j in range(n):
        lines.append(f"h q[{j}];")
        for k in range(j + 1, n):
            lines.append(f"cp(pi/2^{k - j}) q[{k}], q[{j}];")
    for j in range(n // 2):
        lines.append(f"swap q[{j}], q[{n - 1 - j}];")
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("fused", [False, True])
def test_qft_amplitudes_closed_form(T, fused):
    """QFT of a basis state on 10 qubits (most controlled phases act on
    distant qubits): every amplitude is e^{2 pi i x y / N} / sqrt(N)."""
    n, x = 10, 357
    nq, gates = T.parse_qasm(_qft_program(n, x))
    if fused:
        gates = T.fuse(gates, nq)
    m = T.MPS(n, 64)
    m.run_circuit(gates)
    rng = np.random.default_rng(4)
    for y in list(rng.integers(0, 2 ** n, 12)) + [0, 2 ** n - 1]:
        bits = [(int(y) >> (n - 1 - q)) & 1 for q in range(n)]
        want = cmath.exp(2j * math.pi * x * int(y) / 2 ** n) / math.sqrt(2 ** n)
        assert abs(m.amplitude(bits) - want) < 1e-12


@pytest.mark.parametrize("precision,storage,tol", [("fp64", "c128", 1e-12),
                                                   ("bf16x6", "c64", 1e-6)])
def test_fused_heisenberg_vs_unfused_oracle(T, precision, storage, tol):
    """Trotter steps of a Heisenberg chain (three two-qubit gates per bond and
    step, fused into one), n = 12, no truncation: the fused GPU run and the
    unfused oracle run give the same state."""
    n = 12
    nq, gates = T.parse_qasm(W.heisenberg_qasm(n, 4))
    fused = T.fuse(gates, nq)
    assert sum(1 for g in fused if g[1] >= 0) * 3 == sum(1 for g in gates if g[1] >= 0)
    m = T.MPS(n, 64, 0.0, precision=precision, storage=storage)
    m.run_circuit(fused)
    o = O.run_gates(n, 64, 0.0, gates)
    f = mps_fidelity_gpu_vs_oracle(m, o, lambda k: O.OracleMPS(k, 4096))
    assert 1 - f < tol


def test_parsed_fused_circuit_sampled_vs_oracle(T):
    """The whole chain on one circuit: OpenQASM text (distant CNOTs and
    controlled phases, Toffolis, rotations) parsed and fused, run through the
    scheduler with truncation at chi = 16, then sampled; the draws equal the
    oracle's on the same final state."""
    n = 12
    rng = np.random.default_rng(21)
    lines = ['OPENQASM 2.0;', 'include "qelib1.inc";', f"qreg q[{n}];", f"creg c[{n}];"]
    for _ in range(120):
        kind = rng.integers(0, 5)
        a, b, c = (int(x) for x in rng.choice(n, 3, replace=False))
        if kind == 0:
            lines.append(f"u3({rng.uniform(0, 3):.6f}, {rng.uniform(0, 6):.6f}, {rng.uniform(0, 6):.6f}) q[{a}];")
        elif kind == 1:
            lines.append(f"cp({rng.uniform(0, 6):.6f}) q[{a}], q[{b}];")
        elif kind == 2:
            lines.append(f"ccx q[{a}], q[{b}], q[{c}];")
        elif kind == 3:
            lines.append(f"cx q[{a}], q[{b}];")
        else:
            lines.append(f"rzz({rng.uniform(0, 6):.6f}) q[{a}], q[{b}];")
    lines.append("measure q -> c;")
    nq, gates = T.parse_qasm("\n".join(lines) + "\n")
    fused = T.fuse(gates, nq)
    m = T.MPS(n, 16, 1e-10)
    m.run_circuit(fused)
    assert max(m.bond_dims()) == 16  # truncated
    o = O.OracleMPS(n, 4096)
    o.set_state([m.site(q) for q in range(n)], [m.lam(b) for b in range(n - 1)])
    u = rng.random((1500, n))
    bits, logp = m.sample(u)
    rbits, rlogp = o.sample(u)
    assert np.array_equal(bits.cpu().numpy(), rbits)
    assert np.max(np.abs(logp.cpu().numpy() - rlogp)) < 1e-10
