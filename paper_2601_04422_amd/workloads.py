"""Seeded synthetic inputs: gate lists and MPS states.

This module only *makes inputs*.  It holds none of the arithmetic of MPS gate
application (no contraction, no SVD, no truncation); the GPU library and the
CPU oracle both consume what it returns and neither is imported here.

Conventions (shared by every consumer):

* A gate is ``(q0, q1, m)``.  ``q1 == -1`` marks a one-qubit gate with a 2x2
  matrix ``m``.  Otherwise ``m`` is 4x4, row-major, in the basis
  ``|s_q0 s_q1>`` with row index ``2*s_q0 + s_q1`` (``s_q0`` is the major
  bit).  The paper applies a 4x4 gate as a 2x2x2x2 tensor on the two sites
  (Sec. III.A, two-qubit gate); it does not fix a basis order, this is ours.
* Rotation gates follow the textbook definitions R_P(t) = exp(-i t P / 2).
* Brickwork layer ``l`` acts on bonds ``(j, j+1)`` with ``j = l (mod 2)``;
  the paper's brickwork benchmark alternates one- and two-qubit gate layers
  over neighbouring pairs (Sec. V.B, Fig. 5).
* Haar-random U(4): QR of a complex Gaussian matrix with the phases of R's
  diagonal moved into Q (Mezzadri, Notices AMS 54, 2007).

Workload recipes (seeds are fixed so both sides see identical gates):

* ``config_small``   n=10, 10 brickwork layers of Haar U(4), chi_max=32 (seed 1001)
* ``config_wide``    n=64, 20 brickwork layers of Haar U(4), chi_max=256 (seed 1002)
* ``config_chi1024`` n=100, layers of Rx(a), Rz(b) on every qubit then CNOT on
  alternating bonds, chi_max=1024 (seed 1003)
* ``config_ansatz``  n=32, 8 layers of Ry, Rz per qubit + CNOT ladder (seed 1004)
* ``config_batch``   256 brickwork circuits of uneven n, depth and chi_max
  (seed 5000 + c for circuit c)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

Gate = Tuple[int, int, np.ndarray]

# ---------------------------------------------------------------- gate matrices

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI = {"I": I2, "X": PX, "Y": PY, "Z": PZ}


def rot(axis: str, theta: float) -> np.ndarray:
    """R_P(theta) = cos(theta/2) I - i sin(theta/2) P, P in {X, Y, Z}."""
    p = PAULI[axis]
    return math.cos(theta / 2) * I2 - 1j * math.sin(theta / 2) * p


def rx(t: float) -> np.ndarray:
    return rot("X", t)


def ry(t: float) -> np.ndarray:
    return rot("Y", t)


def rz(t: float) -> np.ndarray:
    return rot("Z", t)


def hadamard() -> np.ndarray:
    return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2)


def cnot() -> np.ndarray:
    """CNOT with the control on q0 (the major bit of the 4x4 basis)."""
    return np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                    dtype=np.complex128)


def swap() -> np.ndarray:
    return np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                    dtype=np.complex128)


def haar_u4(rng: np.random.Generator) -> np.ndarray:
    z = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


# ---------------------------------------------------------------- circuits

@dataclass
class Circuit:
    """A gate list grouped in layers of gates on disjoint qubits."""
    n: int
    layers: List[List[Gate]]
    chi_max: int
    cutoff: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    def gates(self) -> List[Gate]:
        return [g for layer in self.layers for g in layer]

    def n2q(self) -> int:
        return sum(1 for g in self.gates() if g[1] >= 0)


def brickwork_haar(n: int, depth: int, seed: int) -> List[List[Gate]]:
    rng = np.random.default_rng(seed)
    layers = []
    for l in range(depth):
        layers.append([(j, j + 1, haar_u4(rng)) for j in range(l % 2, n - 1, 2)])
    return layers


def config_small() -> Circuit:
    return Circuit(10, brickwork_haar(10, 10, 1001), chi_max=32, cutoff=0.0,
                   name="brickwork n=10 depth=10 haar chi_max=32")


def config_wide(depth: int = 20) -> Circuit:
    return Circuit(64, brickwork_haar(64, depth, 1002), chi_max=256, cutoff=1e-10,
                   name=f"brickwork n=64 depth={depth} haar chi_max=256")


def rxrz_cnot_layers(n: int, n_layers: int, seed: int,
                     angle_set: Sequence[float] | None = None) -> List[List[Gate]]:
    """Layer l: Rx(a) then Rz(b) on every qubit, then CNOT(j, j+1) for j = l mod 2.

    Angles are uniform in [0, 2 pi), or drawn uniformly from ``angle_set``
    (used for the basis-state and Clifford special cases).  Returned as three
    disjoint-qubit layers per circuit layer.
    """
    rng = np.random.default_rng(seed)
    out = []
    for l in range(n_layers):
        if angle_set is None:
            a = rng.uniform(0, 2 * math.pi, n)
            b = rng.uniform(0, 2 * math.pi, n)
        else:
            a = rng.choice(np.asarray(angle_set, dtype=np.float64), n)
            b = rng.choice(np.asarray(angle_set, dtype=np.float64), n)
        out.append([(q, -1, rx(a[q])) for q in range(n)])
        out.append([(q, -1, rz(b[q])) for q in range(n)])
        out.append([(j, j + 1, cnot()) for j in range(l % 2, n - 1, 2)])
    return out


def config_chi1024(n_layers: int = 30) -> Circuit:
    return Circuit(100, rxrz_cnot_layers(100, n_layers, 1003), chi_max=1024, cutoff=1e-12,
                   name=f"rx/rz + alternating cnot n=100 layers={n_layers} chi_max=1024")


def ansatz_angles(n: int = 32, n_layers: int = 8, seed: int = 1004) -> np.ndarray:
    """Angles ordered [layer][qubit][Ry, Rz], uniform in [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 2 * math.pi, n_layers * n * 2)


def ansatz_structure(n: int = 32, n_layers: int = 8, ladder: bool = True):
    """Hardware-efficient ansatz as parallel lists.

    Returns ``(gates, param_of_gate, rot_axis)``; ``param_of_gate[g]`` is the
    angle index for rotation gates and -1 for fixed gates, ``rot_axis`` is
    0/1/2 for X/Y/Z.  Layer l: Ry then Rz on every qubit, then the CNOT ladder
    (0,1), (1,2), ..., (n-2, n-1) in sequence.
    """
    qs, ps, axes = [], [], []
    for l in range(n_layers):
        for q in range(n):
            base = (l * n + q) * 2
            qs.append((q, -1)); ps.append(base); axes.append(1)
            qs.append((q, -1)); ps.append(base + 1); axes.append(2)
        if ladder:
            for j in range(n - 1):
                qs.append((j, j + 1)); ps.append(-1); axes.append(-1)
    return qs, ps, axes


def ansatz_gates(angles: np.ndarray, n: int = 32, n_layers: int = 8,
                 ladder: bool = True) -> List[Gate]:
    qs, ps, axes = ansatz_structure(n, n_layers, ladder)
    out = []
    for (q0, q1), p, ax in zip(qs, ps, axes):
        if p >= 0:
            out.append((q0, -1, rot("XYZ"[ax], float(angles[p]))))
        else:
            out.append((q0, q1, cnot()))
    return out


def zz_chain(n: int) -> List[str]:
    """Pauli strings of sum_i Z_i Z_{i+1} on an open chain (char q -> qubit q)."""
    out = []
    for i in range(n - 1):
        s = ["I"] * n
        s[i] = "Z"; s[i + 1] = "Z"
        out.append("".join(s))
    return out


def ghz(n: int) -> List[Gate]:
    """H on qubit 0 then the CNOT chain (0,1), (1,2), ... (Sec. V.A)."""
    return [(0, -1, hadamard())] + [(j, j + 1, cnot()) for j in range(n - 1)]


@dataclass
class BatchCircuit:
    n: int
    depth: int
    chi_max: int
    seed: int
    layers: List[List[Gate]]


def config_batch(n_circuits: int = 256) -> List[BatchCircuit]:
    """Uneven independent brickwork circuits: n in [16, 96], depth in [8, 24],
    chi_max in {32, 64, 128, 256, 512}; circuit c draws from seed 5000 + c."""
    out = []
    for c in range(n_circuits):
        rng = np.random.default_rng(5000 + c)
        n = int(rng.integers(16, 97))
        depth = int(rng.integers(8, 25))
        chi = int(rng.choice([32, 64, 128, 256, 512]))
        layers = brickwork_haar(n, depth, 5000 + c + 100000)
        out.append(BatchCircuit(n, depth, chi, 5000 + c, layers))
    return out


# ---------------------------------------------------------------- synthetic states

def random_isometry(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """rows x cols matrix with orthonormal columns (QR of a complex Gaussian)."""
    z = (rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols)))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def schmidt_profile(rng: np.random.Generator, chi: int, decay: float = 8.0) -> np.ndarray:
    """Decreasing positive weights with sum of squares 1 (a smooth spectrum
    spanning exp(-decay) in amplitude, jittered)."""
    x = np.sort(rng.uniform(0.0, 1.0, chi))
    lam = np.exp(-decay * x)
    lam = np.sort(lam)[::-1]
    return lam / np.linalg.norm(lam)


def flat_schmidt_profile(rng: np.random.Generator, chi: int) -> np.ndarray:
    """Decreasing weights with sum of squares 1 drawn from the quarter-circle
    law p(x) = sqrt(4 - x^2) / pi on [0, 2] (the singular-value law of a large
    square complex Gaussian matrix, i.e. the Schmidt spectrum of a random
    state across a cut with equal dimensions): flat at the top, no gap
    anywhere, unlike the smooth exponential profile.  Rejection sampling."""
    out = np.empty(0)
    while out.size < chi:
        x = rng.uniform(0.0, 2.0, 2 * chi)
        y = rng.uniform(0.0, 2.0, 2 * chi)
        out = np.concatenate([out, x[y * y + x * x <= 4.0]])
    lam = np.sort(out[:chi])[::-1]
    return lam / np.linalg.norm(lam)


def random_canonical_mps(n: int, dims: Sequence[int], seed: int,
                         dtype=np.complex128, profile: str = "smooth"):
    """A left-canonical MPS with prescribed bond dimensions.

    ``dims`` has length n+1 with dims[0] = dims[n] = 1; site q has shape
    (dims[q], 2, dims[q+1]) and satisfies sum_{a,s} conj(A[a,s,b]) A[a,s,b'] =
    delta_{bb'}.  Each inner bond gets a Schmidt-like weight vector: a smooth
    decaying one (``profile="smooth"``) or a random-circuit-like one from the
    quarter-circle law (``profile="flat"``).  Used for full-size inputs that
    would take the CPU hours to reach by simulation.
    """
    rng = np.random.default_rng(seed)
    sites, lams = [], []
    for q in range(n):
        a, b = dims[q], dims[q + 1]
        assert b <= 2 * a, "left-canonical site needs dims[q+1] <= 2*dims[q]"
        u = random_isometry(rng, 2 * a, b)
        sites.append(u.reshape(a, 2, b).astype(dtype))
    prof = {"smooth": schmidt_profile, "flat": flat_schmidt_profile}[profile]
    for q in range(n - 1):
        lams.append(prof(rng, dims[q + 1]))
    return sites, lams


def saturated_dims(n: int, chi_max: int) -> List[int]:
    """Largest left-canonical bond dimensions: min(chi_max, 2^q, 2^(n-q))."""
    return [min(chi_max, 2 ** min(q, n - q)) for q in range(n + 1)]


# ---------------------------------------------------------------- circuits as OpenQASM text

def heisenberg_qasm(n: int, steps: int, dt: float = 0.1, seed: int = 1007) -> str:
    """First-order Trotter steps of a Heisenberg chain with random fields:
    per step rxx, ryy, rzz(2 dt) on every bond (even bonds, then odd) and
    rz(2 dt h_q) on every qubit, h_q uniform in [-1, 1]; starts from the Neel
    state (x on odd qubits).  Three two-qubit gates per bond and step, which
    fusion merges into one."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(-1.0, 1.0, n)
    out = ['OPENQASM 2.0;', 'include "qelib1.inc";', f"qreg q[{n}];", f"creg c[{n}];"]
    out += [f"x q[{q}];" for q in range(1, n, 2)]
    for _ in range(steps):
        for start in (0, 1):
            for j in range(start, n - 1, 2):
                for g in ("rxx", "ryy", "rzz"):
                    out.append(f"{g}({2 * dt!r}) q[{j}], q[{j + 1}];")
        out += [f"rz({float(2 * dt * h[q])!r}) q[{q}];" for q in range(n)]
    out.append("measure q -> c;")
    return "\n".join(out) + "\n"
