"""Independent checkers (numpy only).  They share nothing with the oracle or
the GPU library and are used to pin both.

* ``statevector``      brute-force state vector, index x = sum_q b_q 2^q
                       (direct contraction of the circuit, Sec. II.A eq. 1).
* ``schmidt_values``   singular values of the state reshaped at a cut.
* ``sample_dense``      sequential sampling from a state vector: each qubit's
                       conditional from marginals summed over the full |psi|^2.
* ``pauli_expect_clifford``  <0|U^dag P U|0> by Heisenberg-picture Pauli
                       propagation for Clifford circuits (each gate maps a
                       Pauli string to a signed Pauli string; the map is found
                       numerically from the gate matrix).
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np

_P = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def _axis(n: int, q: int) -> int:
    # C-order reshape to (2,)*n: the last axis is bit 0
    return n - 1 - q


def apply_gate(psi: np.ndarray, n: int, gate) -> np.ndarray:
    q0, q1, m = gate
    t = psi.reshape((2,) * n)
    m = np.asarray(m, dtype=np.complex128)
    if q1 < 0:
        ax = _axis(n, q0)
        t = np.tensordot(m, t, axes=([1], [ax]))
        t = np.moveaxis(t, 0, ax)
    else:
        a0, a1 = _axis(n, q0), _axis(n, q1)
        g4 = m.reshape(2, 2, 2, 2)  # [s0', s1', s0, s1], s0 on q0
        t = np.tensordot(g4, t, axes=([2, 3], [a0, a1]))
        t = np.moveaxis(t, [0, 1], [a0, a1])
    return np.ascontiguousarray(t).reshape(-1)


def statevector(n: int, gates: Iterable) -> np.ndarray:
    psi = zero_state(n)
    for g in gates:
        psi = apply_gate(psi, n, g)
    return psi


def amplitude_index(bits: Sequence[int]) -> int:
    return int(sum(int(b) << q for q, b in enumerate(bits)))


def schmidt_values(psi: np.ndarray, n: int, bond: int) -> np.ndarray:
    """Schmidt coefficients between qubits 0..bond and bond+1..n-1."""
    mat = psi.reshape(2 ** (n - bond - 1), 2 ** (bond + 1))
    return np.linalg.svd(mat, compute_uv=False)


def fidelity_dense(a: np.ndarray, b: np.ndarray) -> float:
    return float(abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))


def expect_dense(psi: np.ndarray, n: int, pauli: str) -> complex:
    phi = psi
    for q, c in enumerate(pauli):
        if c != "I":
            phi = apply_gate(phi, n, (q, -1, _P[c]))
    return complex(np.vdot(psi, phi) / np.vdot(psi, psi))


# ------------------------------------------------------------ Clifford Pauli propagation

def _pauli_decompose(m: np.ndarray, k: int) -> Tuple[complex, str]:
    """m (2^k x 2^k) = c * Q for a single Pauli string Q; returns (c, Q)."""
    best = None
    for labels in itertools.product("IXYZ", repeat=k):
        q = _P[labels[0]]
        for l in labels[1:]:
            q = np.kron(q, _P[l])
        c = np.trace(q.conj().T @ m) / (2 ** k)
        if abs(c) > 1e-9:
            if best is not None:
                raise ValueError("gate is not Clifford: Pauli maps to a sum")
            best = (complex(c), "".join(labels))
    if best is None or abs(abs(best[0]) - 1) > 1e-9:
        raise ValueError("gate is not Clifford")
    return best


def pauli_expect_clifford(n: int, gates: Sequence, pauli: str) -> complex:
    """<0^n| U^dag P U |0^n> with U = g_L ... g_1 (gates in application order)."""
    phase = 1.0 + 0j
    p = list(pauli)
    cache: Dict = {}
    for q0, q1, m in reversed(list(gates)):
        m = np.asarray(m, dtype=np.complex128)
        qs = [q0] if q1 < 0 else [q0, q1]
        local = "".join(p[q] for q in qs)
        if set(local) == {"I"}:
            continue
        key = (m.tobytes(), local)
        if key not in cache:
            pl = _P[local[0]]
            for l in local[1:]:
                pl = np.kron(pl, _P[l])
            cache[key] = _pauli_decompose(m.conj().T @ pl @ m, len(qs))
        c, new = cache[key]
        phase *= c
        for q, l in zip(qs, new):
            p[q] = l
    if any(c in "XY" for c in p):
        return 0.0 + 0j
    return phase


def stabilizer_generator(n: int, gates: Sequence, q: int) -> Tuple[complex, str]:
    """U Z_q U^dag = c * Q for a Clifford U (gates in application order).

    Since U Z_q U^dag stabilises U|0^n>, <psi|Q|psi> = 1/c exactly."""
    phase = 1.0 + 0j
    p = ["I"] * n
    p[q] = "Z"
    cache: Dict = {}
    for q0, q1, m in gates:
        m = np.asarray(m, dtype=np.complex128)
        qs = [q0] if q1 < 0 else [q0, q1]
        local = "".join(p[x] for x in qs)
        if set(local) == {"I"}:
            continue
        key = (m.tobytes(), local)
        if key not in cache:
            pl = _P[local[0]]
            for l in local[1:]:
                pl = np.kron(pl, _P[l])
            cache[key] = _pauli_decompose(m @ pl @ m.conj().T, len(qs))
        c, new = cache[key]
        phase *= c
        for x, l in zip(qs, new):
            p[x] = l
    return phase, "".join(p)


def sample_dense(psi: np.ndarray, n: int, u: np.ndarray):
    """Draw qubits n-1, n-2, ..., 0 in turn; qubit q gets bit 0 when
    u[shot, q] < P(s_q = 0 | bits drawn so far), every marginal summed over
    the whole probability vector.  Returns (bits shots x n, log P(x))."""
    prob = np.abs(psi) ** 2
    total = prob.sum()
    shots = u.shape[0]
    bits = np.zeros((shots, n), dtype=np.uint8)
    logp = np.zeros(shots)
    # marg[q][key]: total probability of the strings whose bits q..n-1 read key
    marg = [prob.reshape(2 ** (n - q), 2 ** q).sum(axis=1) for q in range(n + 1)]
    for shot in range(shots):
        key = 0
        for q in range(n - 1, -1, -1):
            m0, m1 = marg[q][2 * key], marg[q][2 * key + 1]
            b = 0 if u[shot, q] < m0 / (m0 + m1) else 1
            bits[shot, q] = b
            key = 2 * key + b
        logp[shot] = np.log(prob[key] / total)
    return bits, logp
