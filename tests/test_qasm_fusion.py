"""Circuit front end (host code in the library, no GPU): OpenQASM 2.0 parsing
and gate fusion.

The parser is checked against closed forms (the quantum Fourier transform
on basis states, the Toffoli and Fredkin truth tables, a GHZ state) and
against identities between gates that follow from their definitions; fusion
is checked to keep the circuit's unitary (brute-force state vectors) and to
reach the gate counts its rules imply.
"""
import cmath
import math

import numpy as np
import pytest

from checkers import apply_gate, statevector
from paper_2601_04422_amd import tnsim as T
from paper_2601_04422_amd import workloads as W

HDR = 'OPENQASM 2.0;\ninclude "qelib1.inc";\n'


def unitary(n, gates):
    cols = []
    for x in range(2 ** n):
        psi = np.zeros(2 ** n, dtype=np.complex128)
        psi[x] = 1.0
        for g in gates:
            psi = apply_gate(psi, n, g)
        cols.append(psi)
    return np.array(cols).T


def parse_unitary(body, n):
    nq, gates = T.parse_qasm(HDR + f"qreg q[{n}];\n" + body)
    assert nq == n
    return unitary(n, gates)


def qft_text(n):
    lines = []
    for j in range(n):
        lines.append(f"h q[{j}];")
        for k in range(j + 1, n):
            lines.append(f"cp(pi/2^{k - j}) q[{k}], q[{j}];")
    for j in range(n // 2):
        lines.append(f"swap q[{j}], q[{n - 1 - j}];")
    return "\n".join(lines)


def test_qft_closed_form():
    """QFT on basis states: |x> -> sum_y e^{2 pi i x y / N} |y> / sqrt(N), with
    qubit 0 the most significant bit of x and y (the textbook circuit)."""
    n = 5
    N = 2 ** n
    U = parse_unitary(qft_text(n), n)

    def msb(idx):  # integer read with qubit 0 as the most significant bit
        return sum(((idx >> q) & 1) << (n - 1 - q) for q in range(n))

    want = np.array([[cmath.exp(2j * math.pi * msb(x) * msb(y) / N) / math.sqrt(N)
                      for x in range(N)] for y in range(N)])
    assert np.max(np.abs(U - want)) < 1e-12


def test_toffoli_and_fredkin_truth_tables():
    U = parse_unitary("ccx q[0], q[1], q[2];", 3)
    for x in range(8):
        b0, b1, b2 = x & 1, (x >> 1) & 1, (x >> 2) & 1
        y = b0 | (b1 << 1) | ((b2 ^ (b0 & b1)) << 2)
        col = np.zeros(8)
        col[y] = 1
        assert np.max(np.abs(U[:, x] - col)) < 1e-12
    U = parse_unitary("cswap q[2], q[0], q[1];", 3)
    for x in range(8):
        b0, b1, b2 = x & 1, (x >> 1) & 1, (x >> 2) & 1
        if b2:
            b0, b1 = b1, b0
        col = np.zeros(8)
        col[b0 | (b1 << 1) | (b2 << 2)] = 1
        assert np.max(np.abs(U[:, x] - col)) < 1e-12


def test_barrier_measure_and_classical_registers_are_skipped():
    nq, gates = T.parse_qasm(HDR + "qreg a[2];\ncreg c[2];\nqreg b[1];\n"
                             "h a[0];\nbarrier a, b;\ncx a[0], b[0];\nmeasure a -> c;\n"
                             "measure b[0] -> c[1];\n// a comment\n/* and\n another */\n")
    assert nq == 3
    assert [(g[0], g[1]) for g in gates] == [(0, -1), (0, 2)]


def test_ghz_state():
    nq, gates = T.parse_qasm(HDR + "qreg a[2];\nqreg b[3];\n"
                             "h a[0];\ncx a[0], a[1];\ncx a[1], b[0];\ncx b[0], b[1];\ncx b[1], b[2];\n")
    assert nq == 5
    psi = statevector(5, gates)
    want = np.zeros(32)
    want[0] = want[31] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - want)) < 1e-14


def test_broadcast():
    nq, gates = T.parse_qasm(HDR + "qreg q[3];\nqreg r[3];\nx q;\ncx q, r;\n")
    assert [(g[0], g[1]) for g in gates] == [(0, -1), (1, -1), (2, -1), (0, 3), (1, 4), (2, 5)]
    psi = statevector(6, gates)
    assert abs(psi[63] - 1) < 1e-14


GATE_IDENTITIES = [
    # (qasm a, qasm b, n): the two programs are the same unitary up to a global phase
    ("u3(pi/2, 0, pi) q[0];", "h q[0];", 1),
    ("u2(0, pi) q[0];", "h q[0];", 1),
    ("sx q[0]; sx q[0];", "x q[0];", 1),
    ("sxdg q[0]; sx q[0];", "id q[0];", 1),
    ("s q[0]; s q[0];", "z q[0];", 1),
    ("t q[0]; t q[0];", "s q[0];", 1),
    ("sdg q[0]; s q[0];", "id q[0];", 1),
    ("tdg q[0]; t q[0];", "i q[0];", 1),
    ("h q[0]; rz(0.7) q[0]; h q[0];", "rx(0.7) q[0];", 1),
    ("rx(pi) q[0];", "x q[0];", 1),
    ("ry(pi) q[0];", "y q[0];", 1),
    ("rz(0.4) q[0];", "u1(0.4) q[0];", 1),
    ("p(0.4) q[0];", "u1(0.4) q[0];", 1),
    ("U(0.3, 0.2, 0.1) q[0];", "rz(0.1) q[0]; ry(0.3) q[0]; rz(0.2) q[0];", 1),
    ("u(0.3, 0.2, 0.1) q[0];", "u3(0.3, 0.2, 0.1) q[0];", 1),
    ("h q[1]; cx q[0], q[1]; h q[1];", "cz q[0], q[1];", 2),
    ("cz q[0], q[1];", "cz q[1], q[0];", 2),
    ("sdg q[1]; cx q[0], q[1]; s q[1];", "cy q[0], q[1];", 2),
    ("cx q[0], q[1]; cx q[1], q[0]; cx q[0], q[1];", "swap q[0], q[1];", 2),
    ("CX q[0], q[1];", "cx q[0], q[1];", 2),
    ("cx q[0], q[1]; rz(0.9) q[1]; cx q[0], q[1];", "rzz(0.9) q[0], q[1];", 2),
    ("h q[0]; h q[1]; rzz(0.9) q[0], q[1]; h q[0]; h q[1];", "rxx(0.9) q[0], q[1];", 2),
    ("rx(pi/2) q[0]; rx(pi/2) q[1]; rzz(0.9) q[0], q[1]; rx(-pi/2) q[0]; rx(-pi/2) q[1];",
     "ryy(0.9) q[0], q[1];", 2),
    ("cp(0.5) q[0], q[1];", "cu1(0.5) q[1], q[0];", 2),
    ("crz(0.5) q[0], q[1];", "rz(0.25) q[1]; cx q[0], q[1]; rz(-0.25) q[1]; cx q[0], q[1];", 2),
    ("cry(0.5) q[0], q[1];", "ry(0.25) q[1]; cx q[0], q[1]; ry(-0.25) q[1]; cx q[0], q[1];", 2),
    ("crx(0.5) q[0], q[1];", "h q[1]; crz(0.5) q[0], q[1]; h q[1];", 2),
    ("ch q[0], q[1];", "ry(-pi/4) q[1]; cz q[0], q[1]; ry(pi/4) q[1];", 2),
    ("csx q[0], q[1];", "h q[1]; cp(pi/2) q[0], q[1]; h q[1];", 2),
    ("cu3(0.3, 0.2, 0.1) q[0], q[1];", "cu(0.3, 0.2, 0.1, 0) q[0], q[1];", 2),
    ("cu(0.3, 0.2, 0.1, 0.6) q[0], q[1];", "cu3(0.3, 0.2, 0.1) q[0], q[1]; p(0.6) q[0];", 2),
    ("rz(-pi/4 + 2*0.5^2) q[0];", "rz(sqrt(0.0625) + ln(exp(0.0)) - pi/4 + 0.25) q[0];", 1),
    ("gate my(a, b) x, y { rx(a) x; cx x, y; ry(b/2) y; }\nmy(0.3, 0.8) q[1], q[0];",
     "rx(0.3) q[1]; cx q[1], q[0]; ry(0.4) q[0];", 2),
    ("gate inner(t) z { rz(t) z; }\ngate outer(t) a, b { inner(2*t) b; cz a, b; }\nouter(0.2) q[0], q[1];",
     "rz(0.4) q[1]; cz q[0], q[1];", 2),
]


def _same_up_to_phase(a, b):
    k = np.argmax(np.abs(b))
    ph = a.flat[k] / b.flat[k]
    return abs(abs(ph) - 1) < 1e-12 and np.max(np.abs(a - ph * b)) < 1e-12


@pytest.mark.parametrize("a,b,n", GATE_IDENTITIES)
def test_gate_identities(a, b, n):
    assert _same_up_to_phase(parse_unitary(a, n), parse_unitary(b, n))


def test_definitions_exact_phases():
    """The global phases are those of the definitions: R_P(t) = exp(-itP/2)
    and p(l) = diag(1, e^{il}) (no phase freedom here)."""
    U = parse_unitary("rz(0.6) q[0];", 1)
    assert np.max(np.abs(U - np.diag([cmath.exp(-0.3j), cmath.exp(0.3j)]))) < 1e-15
    U = parse_unitary("p(0.6) q[0];", 1)
    assert np.max(np.abs(U - np.diag([1, cmath.exp(0.6j)]))) < 1e-15
    U = parse_unitary("rx(0.6) q[0];", 1)
    c, s = math.cos(0.3), math.sin(0.3)
    assert np.max(np.abs(U - np.array([[c, -1j * s], [-1j * s, c]]))) < 1e-15


@pytest.mark.parametrize("text,msg", [
    ("qreg q[2];\nfoo q[0];", "unknown gate"),
    ("qreg q[2];\ncx q[0];", "qubits"),
    ("qreg q[2];\nh q[2];", "out of range"),
    ("qreg q[2];\nreset q[0];", "not supported"),
    ("qreg q[2];\ncx q[0], q[0];", "twice"),
    ("qreg q[2];\nrx(1 +) q[0];", "expression"),
    ("qreg q[2];\nh q[0]", "expected"),
    ("qreg q[2];\nqreg r[3];\ncx q, r;", "different sizes"),
    ("qreg q[2];\nrx(theta) q[0];", "unknown parameter"),
    ("qreg q[2];\nh q[0]; @", "unexpected character"),
    ("qreg q[1];\nrx(" + "(" * 400 + "1" + ")" * 400 + ") q[0];", "nested too deeply"),
    ("qreg q[1];\ngate g a { g a; }\ng q[0];", "nested too deeply"),
    ("qreg q[1];\nopaque g a;", "not supported"),
    ("OPENQASM 3.0;\nqreg q[1];", "OpenQASM 2"),
    ("qreg q[1];\nrx(1/0) q[0];", "not finite"),
    ("qreg q[1];\nrz(1e999) q[0];", "not finite"),
])
def test_errors(text, msg):
    with pytest.raises(T.TnsimError) as e:
        T.parse_qasm(HDR + text)
    assert e.value.code == T.E_ARG
    assert msg in str(e.value)
    assert "line" in str(e.value)


def test_capacity_query():
    import ctypes as C

    text = (HDR + "qreg q[3];\nh q;\ncx q[0], q[1];\n").encode()
    n, nq = C.c_int32(), C.c_int32()
    arr = np.zeros(2, dtype=T.GATE_DTYPE)
    st = T.lib().tnsim_qasm_parse(text, arr.ctypes.data, 2, C.byref(n), C.byref(nq), None, 0)
    assert st == T.E_CAPACITY and n.value == 4 and nq.value == 3


# ---------------------------------------------------------------- fusion

def _random_circuit(n, count, seed, local=False):
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(count):
        if rng.random() < 0.5:
            q = int(rng.integers(0, n))
            gates.append((q, -1, W.rot("XYZ"[int(rng.integers(0, 3))], rng.uniform(0, 6.3))))
        else:
            if local:
                a = int(rng.integers(0, n - 1))
                a, b = (a, a + 1) if rng.random() < 0.5 else (a + 1, a)
            else:
                a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            gates.append((a, b, W.haar_u4(rng) if rng.random() < 0.7 else W.cnot()))
    return gates


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fusion_keeps_the_unitary(seed):
    n = 6
    gates = _random_circuit(n, 80, seed)
    fused = T.fuse(gates, n)
    assert len(fused) < len(gates)
    assert np.max(np.abs(unitary(n, fused) - unitary(n, gates))) < 1e-12


def test_fusion_counts():
    """Rules: one-qubit gates go into the neighbouring two-qubit gate; a
    two-qubit gate directly after another on the same pair (either order)
    merges; a qubit without two-qubit gates keeps one fused gate."""
    n = 4
    h, cx = W.hadamard(), W.cnot()
    gates = [(0, -1, h), (1, -1, h), (0, 1, cx), (0, -1, h), (1, 0, cx), (1, -1, h),
             (0, 1, cx), (2, -1, h), (2, -1, h), (2, -1, h)]
    fused = T.fuse(gates, n)
    assert [(g[0], g[1]) for g in fused] == [(0, 1), (2, -1)]
    assert np.max(np.abs(unitary(n, fused) - unitary(n, gates))) < 1e-12
    # a gate on another qubit pair in between stops the merge
    gates = [(0, 1, cx), (1, 2, cx), (0, 1, cx)]
    assert len(T.fuse(gates, 3)) == 3


def test_fusion_of_the_benchmark_circuit():
    """The chi=1024 benchmark circuit (Rx, Rz on every qubit, then a CNOT
    brickwork layer): every rotation folds into a CNOT, so the fused circuit
    is exactly its two-qubit gates."""
    n, L = 10, 6
    gates = [g for sub in W.config_chi1024(L).layers for g in sub]  # n = 100
    # the same structure at n = 10, small enough for the unitary
    rng = np.random.default_rng(1)
    small = []
    for l in range(L):
        for q in range(n):
            small.append((q, -1, W.rx(rng.uniform(0, 6.28))))
            small.append((q, -1, W.rz(rng.uniform(0, 6.28))))
        for j in range(l % 2, n - 1, 2):
            small.append((j, j + 1, W.cnot()))
    n2 = sum(1 for g in small if g[1] >= 0)
    fused = T.fuse(small, n)
    assert len(fused) == n2 and all(g[1] >= 0 for g in fused)
    assert np.max(np.abs(unitary(n, fused) - unitary(n, small))) < 1e-12
    f100 = T.fuse(gates, 100)
    assert len(f100) == sum(1 for g in gates if g[1] >= 0)


def test_fusion_of_a_parsed_circuit():
    n = 5
    nq, gates = T.parse_qasm(HDR + f"qreg q[{n}];\n" + qft_text(n) + "\nccx q[0], q[2], q[4];\n")
    fused = T.fuse(gates, nq)
    assert len(fused) < len(gates)
    assert np.max(np.abs(unitary(n, fused) - unitary(n, gates))) < 1e-12


def test_fusion_errors():
    with pytest.raises(T.TnsimError):
        T.fuse([(0, 3, W.cnot())], 3)
    with pytest.raises(T.TnsimError):
        T.fuse([(1, 1, W.cnot())], 3)
    assert T.fuse([], 3) == []
