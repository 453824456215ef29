"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names the part of the oracle it pins.  None of them compares the
oracle with itself: expected values come from closed forms, a brute-force
state vector (numpy), numpy's SVD, Clifford Pauli propagation, or the golden
fixtures under tests/golden/ (each citing the paper).
"""
import math
import os

import numpy as np
import pytest

from checkers import (amplitude_index, expect_dense, fidelity_dense, pauli_expect_clifford,
                      sample_dense, schmidt_values, stabilizer_generator, statevector)
from oracle import oracle as O
from paper_2601_04422_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return rows


# ---------------------------------------------------------------- P1: 1q gates

def test_product_state_closed_forms():
    """Pins init |0...0> and the one-qubit contraction (eq. 3)."""
    rows = _read_table("product_state.txt")
    n = 3 * len(rows)
    m = O.OracleMPS(n, 4)
    for r, (th, ph, al) in enumerate(rows):
        m.apply((3 * r, -1, W.ry(th)))
        m.apply((3 * r, -1, W.rz(ph)))
        m.apply((3 * r + 1, -1, W.rx(al)))
    for r, (th, ph, al) in enumerate(rows):
        def e(q, c):
            s = ["I"] * n
            s[q] = c
            return m.expect("".join(s))
        assert abs(e(3 * r, "Z") - math.cos(th)) < 1e-14
        assert abs(e(3 * r, "X") - math.sin(th) * math.cos(ph)) < 1e-14
        assert abs(e(3 * r, "Y") - math.sin(th) * math.sin(ph)) < 1e-14
        assert abs(e(3 * r + 1, "Z") - math.cos(al)) < 1e-14
        assert abs(e(3 * r + 1, "Y") + math.sin(al)) < 1e-14
        assert abs(e(3 * r + 1, "X")) < 1e-14
        assert abs(e(3 * r + 2, "Z") - 1.0) < 1e-14  # untouched qubit stays |0>
    assert list(m.bond_dims()) == [1] * (n - 1)


# ---------------------------------------------------------------- P2: untruncated circuits

def test_small_brickwork_matches_statevector():
    """Pins a3-a8 without truncation: the n=10, depth-10 Haar brickwork at
    chi_max=32 (no cut possible) against the brute-force state vector."""
    cfg = W.config_small()
    m = O.OracleMPS(cfg.n, cfg.chi_max, cfg.cutoff)
    m.run_layers(cfg.layers)
    ref = statevector(cfg.n, cfg.gates())
    got = m.statevector()
    assert np.max(np.abs(got - ref)) < 1e-12
    rng = np.random.default_rng(7)
    for _ in range(20):
        bits = rng.integers(0, 2, cfg.n)
        assert abs(m.amplitude(bits) - ref[amplitude_index(bits)]) < 1e-12
    assert m.stats()["sum_eps"] < 1e-24


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_random_circuits_with_1q_and_reversed_gates(seed):
    """Mixed 1q/2q gates, gates given as (q, q-1), odd n: brute force."""
    rng = np.random.default_rng(seed)
    n = 7
    gates = []
    for _ in range(40):
        if rng.random() < 0.4:
            q = int(rng.integers(0, n))
            gates.append((q, -1, W.rot("XYZ"[int(rng.integers(0, 3))], rng.uniform(0, 6.3))))
        else:
            j = int(rng.integers(0, n - 1))
            g = W.haar_u4(rng)
            gates.append((j, j + 1, g) if rng.random() < 0.5 else (j + 1, j, g))
    m = O.run_gates(n, 64, 0.0, gates)
    ref = statevector(n, gates)
    assert np.max(np.abs(m.statevector() - ref)) < 1e-12


# ---------------------------------------------------------------- P3: GHZ golden

def test_ghz_golden():
    """Sec. V.A: GHZ = (|0..0> + |1..1>)/sqrt(2) with chi = 2 on every bond."""
    for n, a0, a1, chi in _read_table("ghz.txt"):
        n = int(n)
        m = O.run_gates(n, 64, 0.0, W.ghz(n))
        assert abs(m.amplitude([0] * n) - a0) < 1e-14
        assert abs(m.amplitude([1] * n) - a1) < 1e-14
        bits = [0] * n
        bits[n // 2] = 1
        assert abs(m.amplitude(bits)) < 1e-14
        assert max(m.bond_dims()) <= chi
        assert int(max(m.bond_dims())) == int(chi)


# ---------------------------------------------------------------- P4, P5: spectra, norms

def test_lambda_are_schmidt_values_and_norm():
    """lambda_q equals the Schmidt spectrum of the exact state at cut q (P4);
    <psi|psi> = 1 and sum lambda^2 = 1 (P5)."""
    n = 8
    layers = W.brickwork_haar(n, 7, 2024)
    gates = [g for l in layers for g in l]
    m = O.OracleMPS(n, 256, 0.0)
    m.run_layers(layers)
    psi = statevector(n, gates)
    for b in range(n - 1):
        ref = schmidt_values(psi, n, b)
        lam = m.lam(b)
        ref = ref[: lam.size]
        assert np.max(np.abs(lam - ref)) < 1e-12
        assert abs(np.sum(lam ** 2) - 1) < 1e-12
    assert abs(m.norm2() - 1) < 1e-12
    # left-canonical sites (the gauge reading): sum_{a,s} conj(A) A = I
    for q in range(n - 1):
        a = m.site(q)
        mat = a.reshape(-1, a.shape[2])
        assert np.max(np.abs(mat.conj().T @ mat - np.eye(a.shape[2]))) < 1e-12


# ---------------------------------------------------------------- P6: truncation weight

def test_truncation_error_equals_discarded_weight():
    """On an exactly canonical state one truncated gate gives
    1 - F(exact, truncated) = eps and ||psi_exact - N psi_trunc||^2 = eps."""
    n = 8
    layers = W.brickwork_haar(n, 6, 77)
    exact = O.OracleMPS(n, 256, 0.0)
    exact.run_layers(layers)
    sites = [exact.site(q) for q in range(n)]
    lams = [exact.lam(b) for b in range(n - 1)]
    rng = np.random.default_rng(5)
    g = W.haar_u4(rng)
    bond = 3
    full = O.OracleMPS(n, 256, 0.0)
    full.set_state(sites, lams)
    full.apply_2q(bond, bond + 1, g)
    chi_before = exact.bond_dims()[bond]
    for chi_cut in (chi_before // 2, chi_before // 4, 1):
        tr = O.OracleMPS(n, chi_cut, 0.0)
        tr.set_state(sites, lams)
        assert tr.apply_2q(bond, bond + 1, g) == O.OK
        eps = tr.stats()["last_eps"]
        assert eps > 1e-6
        psi_e = full.statevector()
        psi_t = tr.statevector()
        f = fidelity_dense(psi_e, psi_t)
        assert abs((1 - f) - eps) < 1e-12
        assert abs(np.sum(np.abs(psi_e - math.sqrt(1 - eps) * psi_t) ** 2) - eps) < 1e-12
        assert abs(np.sum(tr.lam(bond) ** 2) - 1) < 1e-12  # kept weights renormalised
        # discarded weight from the exact Schmidt spectrum at that bond
        lam_full = full.lam(bond)
        assert abs(np.sum(lam_full[chi_cut:] ** 2) - eps) < 1e-12


# ---------------------------------------------------------------- P7: SVD

@pytest.mark.parametrize("shape", [(6, 6), (16, 8), (8, 16), (64, 64), (40, 128), (130, 70)])
def test_jacobi_svd_against_numpy(shape):
    """The oracle's Jacobi SVD against numpy's LAPACK SVD: singular values,
    orthonormal U, and U U^H M = M (U spans the column space)."""
    rng = np.random.default_rng(sum(shape))
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    u, s, sweeps = O.svd(a)
    ref = np.linalg.svd(a, compute_uv=False)
    assert sweeps > 0
    assert np.max(np.abs(s - ref)) / ref[0] < 1e-13
    r = min(shape)
    assert np.max(np.abs(u.conj().T @ u - np.eye(r))) < 1e-13
    assert np.linalg.norm(a - u @ (u.conj().T @ a)) / np.linalg.norm(a) < 1e-13
    # sigma_j = || u_j^H M ||
    assert np.max(np.abs(np.linalg.norm(u.conj().T @ a, axis=1) - s)) / s[0] < 1e-13


def test_jacobi_svd_graded_and_rank_deficient():
    rng = np.random.default_rng(9)
    q1 = W.random_isometry(rng, 50, 50)
    q2 = W.random_isometry(rng, 50, 50)
    sig = np.logspace(0, -12, 50)
    a = (q1 * sig) @ q2.conj().T
    u, s, _ = O.svd(a)
    # forming a in floating point perturbs it by ~1e-16 * ||a||: absolute accuracy
    # at that level for all values, relative accuracy for the values well above it
    assert np.max(np.abs(s - sig)) < 1e-13
    big = sig > 1e-6
    assert np.max(np.abs(s[big] - sig[big]) / sig[big]) < 1e-9
    # rank 3 in a 20 x 20 matrix
    b = W.random_isometry(rng, 20, 3) @ W.random_isometry(rng, 20, 3).conj().T
    _, s2, _ = O.svd(b)
    assert np.allclose(s2[:3], 1.0, atol=1e-13) and np.max(s2[3:]) < 1e-13


def test_noconvergence_is_reported():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32))
    with pytest.raises(O.OracleError) as e:
        O.svd(a, max_sweeps=1)
    assert e.value.code == O.E_NOCONV
    # a sweep with no rotation is needed to stop, so one sweep never suffices
    m = O.OracleMPS(4, 16, 0.0, max_sweeps=1)
    assert m.apply_2q(1, 2, W.haar_u4(rng)) == O.E_NOCONV
    assert list(m.bond_dims()) == [1, 1, 1]  # state left unchanged


# ---------------------------------------------------------------- truncation rule

def test_truncation_rule():
    # sigma^2 = [9/16, 1/4, 1/16, 1/16, 1/16]: dyadic, so W = 1 and every tail is exact
    s = np.array([0.75, 0.5, 0.25, 0.25, 0.25])
    # a tail exactly equal to cutoff * W is discarded (tail <= cutoff * W)
    assert O.truncation(s, 10, 99, 0.0625)[0] == 4
    assert O.truncation(s, 10, 99, 0.0625 - 1e-12)[0] == 5
    assert O.truncation(s, 10, 99, 0.125)[0] == 3
    k, eps, nrm = O.truncation(s, 10, 2, 0.0)
    assert k == 2 and abs(eps - 0.1875) < 1e-15 and abs(nrm - math.sqrt(0.8125)) < 1e-15
    assert O.truncation(s, 10, 99, 10.0)[0] == 1  # k >= 1
    # numerical-zero floor: sigma^2 <= rows * 2^-53 * sigma_1^2
    z = np.array([1.0, 1e-3, 1e-9])
    assert O.truncation(z, 4, 99, 0.0)[0] == 2
    assert O.truncation(np.array([1.0, 3e-8]), 2, 99, 0.0)[0] == 2
    assert O.truncation(np.array([1.0, 1e-8]), 2, 99, 0.0)[0] == 1


# ---------------------------------------------------------------- P8: layer order

def test_layer_order_independence():
    n = 10
    layers = W.brickwork_haar(n, 6, 31)
    a = O.OracleMPS(n, 8, 1e-10)
    b = O.OracleMPS(n, 8, 1e-10)
    rng = np.random.default_rng(0)
    for layer in layers:
        assert a.apply_layer(layer) == O.OK
        perm = rng.permutation(len(layer))
        assert b.apply_layer([layer[i] for i in perm]) == O.OK
    for q in range(n):
        assert np.array_equal(a.site(q), b.site(q))
    assert a.stats()["sum_eps"] > 0  # the check runs with truncation active


def test_layer_validation():
    m = O.OracleMPS(6, 8)
    g = W.cnot()
    assert m.apply_layer([(0, 1, g), (1, 2, g)]) == O.E_OVERLAP
    assert m.apply_layer([(0, 2, g)]) == O.E_NONLOCAL
    assert m.apply_layer([(5, 6, g)]) == O.E_ARG
    assert m.apply_layer([(0, -1, W.hadamard()), (0, 1, g)]) == O.E_OVERLAP
    assert list(m.bond_dims()) == [1] * 5  # state unchanged


# ---------------------------------------------------------------- P9: large-n structure

def test_basis_state_circuit_n100():
    """Rx in {0, pi}: CNOTs act as reversible logic, chi stays 1, |amp| = 1."""
    n, nl = 100, 12
    layers = W.rxrz_cnot_layers(n, nl, 3, angle_set=[0.0, math.pi])
    m = O.OracleMPS(n, 1024, 1e-12)
    m.run_layers(layers)
    bits = [0] * n
    for layer in layers:
        for q0, q1, g in layer:
            if q1 < 0:
                if abs(abs(g[0, 1]) - 1) < 1e-12:  # Rx(pi) flips, Rz keeps
                    bits[q0] ^= 1
            elif bits[q0]:
                bits[q1] ^= 1
    assert max(m.bond_dims()) == 1
    assert abs(abs(m.amplitude(bits)) - 1) < 1e-12
    for q in (0, 17, 50, 99):
        s = ["I"] * n
        s[q] = "Z"
        assert abs(m.expect("".join(s)).real - (1 - 2 * bits[q])) < 1e-12


def test_clifford_circuit_against_pauli_propagation():
    """Angles in multiples of pi/2: a stabiliser state; <Z_i>, <Z_i Z_i+1>
    in {0, +-1} from Pauli propagation (no truncation reached)."""
    n, nl = 40, 8
    layers = W.rxrz_cnot_layers(n, nl, 4, angle_set=[0.0, math.pi / 2, math.pi, 3 * math.pi / 2])
    gates = [g for l in layers for g in l]
    m = O.OracleMPS(n, 1024, 1e-12)
    m.run_layers(layers)
    checked_nonzero = 0
    for q in range(0, n - 2):
        for ops in (("Z",), ("Z", "Z"), ("X", "X"), ("Y", "Z"), ("X", "Y", "Z"), ("Z", "X", "Z")):
            s = ["I"] * n
            for k, c in enumerate(ops):
                s[q + k] = c
            s = "".join(s)
            ref = pauli_expect_clifford(n, gates, s)
            got = m.expect(s)
            assert abs(got - ref) < 1e-12, (s, got, ref)
            checked_nonzero += abs(ref) > 0.5
    # stabiliser generators U Z_q U^dag have expectation exactly 1/c
    for q in range(0, n, 5):
        c, pstr = stabilizer_generator(n, gates, q)
        assert abs(m.expect(pstr) - 1 / c) < 1e-12, (q, pstr)
        assert abs(pauli_expect_clifford(n, gates, pstr) - 1 / c) < 1e-12
        checked_nonzero += 1
    assert checked_nonzero >= 3
    assert max(m.bond_dims()) >= 4


# ---------------------------------------------------------------- P10: gradients

def test_ansatz_closed_form_and_parameter_shift():
    """No CNOTs: L = sum_i cos(t_i) cos(t_{i+1}) over the Ry angles, dL/dRz = 0."""
    n = 6
    angles = W.ansatz_angles(n, 1, 42)
    gates = W.ansatz_gates(angles, n, 1, ladder=False)
    paulis = W.zz_chain(n)
    coeffs = [1.0] * len(paulis)
    m = O.run_gates(n, 16, 0.0, gates)
    th = angles[0::2]
    ref = sum(math.cos(th[i]) * math.cos(th[i + 1]) for i in range(n - 1))
    assert abs(O.loss_pauli_sum(m, paulis, coeffs) - ref) < 1e-13
    g = O.parameter_shift(lambda a: W.ansatz_gates(a, n, 1, ladder=False), angles, n, 16, 0.0,
                          paulis, coeffs)
    gref = np.zeros_like(angles)
    for i in range(n):
        nb = (math.cos(th[i - 1]) if i > 0 else 0.0) + (math.cos(th[i + 1]) if i < n - 1 else 0.0)
        gref[2 * i] = -math.sin(th[i]) * nb
    assert np.max(np.abs(g - gref)) < 1e-12


def test_parameter_shift_matches_finite_differences_with_cnots():
    n, nl = 5, 2
    angles = W.ansatz_angles(n, nl, 3)
    paulis = W.zz_chain(n)
    coeffs = [1.0] * len(paulis)
    make = lambda a: W.ansatz_gates(a, n, nl)
    g = O.parameter_shift(make, angles, n, 64, 0.0, paulis, coeffs)
    h = 1e-5
    fd = np.zeros_like(angles)
    for p in range(angles.size):
        vals = []
        for sgn in (1, -1):
            a = angles.copy()
            a[p] += sgn * h
            vals.append(O.loss_pauli_sum(O.run_gates(n, 64, 0.0, make(a)), paulis, coeffs))
        fd[p] = (vals[0] - vals[1]) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-8
    # and the loss itself against the brute-force state vector
    psi = statevector(n, make(angles))
    ref = sum(expect_dense(psi, n, p).real for p in paulis)
    assert abs(O.loss_pauli_sum(O.run_gates(n, 64, 0.0, make(angles)), paulis, coeffs) - ref) < 1e-12


# ---------------------------------------------------------------- non-local gates (SWAP chains)

def nonlocal_circuit(n, count, seed):
    """Random circuit of one-qubit rotations and Haar two-qubit gates on
    arbitrary qubit pairs, both orders."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(count):
        if rng.random() < 0.3:
            q = int(rng.integers(0, n))
            gates.append((q, -1, W.rot("XYZ"[int(rng.integers(0, 3))], rng.uniform(0, 6.3))))
        else:
            a, b = rng.choice(n, 2, replace=False)
            gates.append((int(a), int(b), W.haar_u4(rng)))
    return gates


def test_nonlocal_gates_match_statevector():
    """Sec. IV.A: a gate on distant qubits is applied through SWAP gates that
    bring the qubits together and then move them back; without truncation the
    state must equal the brute-force state vector with the gate acting on the
    named qubits directly."""
    n = 7
    gates = nonlocal_circuit(n, 30, 314)
    assert any(g[1] >= 0 and abs(g[0] - g[1]) > 1 for g in gates)
    assert any(g[1] >= 0 and g[0] - g[1] > 1 for g in gates)
    m = O.run_gates(n, 256, 0.0, gates)
    ref = statevector(n, gates)
    got = m.statevector()
    assert np.max(np.abs(got - ref)) < 1e-12


def test_nonlocal_ghz_closed_form():
    """H on qubit 0, then CNOTs from qubit 0 to every other qubit in a
    scrambled order (all but one non-local): the GHZ state, chi = 2."""
    n = 20
    rng = np.random.default_rng(5)
    gates = [(0, -1, W.hadamard())] + [(0, int(j), W.cnot()) for j in rng.permutation(np.arange(1, n))]
    m = O.run_gates(n, 16, 0.0, gates)
    assert abs(m.amplitude([0] * n) - 1 / math.sqrt(2)) < 1e-14
    assert abs(m.amplitude([1] * n) - 1 / math.sqrt(2)) < 1e-14
    assert int(max(m.bond_dims())) == 2


# ---------------------------------------------------------------- P: perfect sampling

def _assert_same_draws(bits, ref_bits, u, psi, n, margin=1e-9):
    """Bits must agree wherever the draw was not a near-tie of u with the
    conditional probability (none is expected with these seeds)."""
    prob = np.abs(psi) ** 2
    marg = [prob.reshape(2 ** (n - q), 2 ** q).sum(axis=1) for q in range(n + 1)]
    for shot in np.nonzero((bits != ref_bits).any(axis=1))[0]:
        key = 0
        for q in range(n - 1, -1, -1):
            m0, m1 = marg[q][2 * key], marg[q][2 * key + 1]
            if bits[shot, q] != ref_bits[shot, q]:
                assert abs(u[shot, q] - m0 / (m0 + m1)) < margin, (shot, q)
                break
            key = 2 * key + int(ref_bits[shot, q])


def test_sampling_matches_brute_force():
    """Sec. III.A perfect sampling: with the same uniforms, every drawn string
    equals sequential sampling from the brute-force state vector, and the
    returned log-probability is log(|<x|psi>|^2)."""
    n = 8
    gates = nonlocal_circuit(n, 40, 2718)
    m = O.run_gates(n, 256, 0.0, gates)
    psi = statevector(n, gates)
    u = np.random.default_rng(17).random((300, n))
    bits, logp = m.sample(u)
    ref_bits, ref_logp = sample_dense(psi, n, u)
    assert np.array_equal(bits, ref_bits)
    assert np.max(np.abs(logp - ref_logp)) < 1e-10
    assert len({tuple(b) for b in bits}) > 100  # a spread distribution, not one string


def test_sampling_in_any_gauge():
    """The marginals use the left block's Gram matrix, so a state stored in a
    non-canonical gauge (random invertible matrices on every bond) and with
    a norm other than 1 samples exactly like the canonical one."""
    n = 7
    gates = nonlocal_circuit(n, 30, 99)
    m = O.run_gates(n, 256, 0.0, gates)
    rng = np.random.default_rng(3)
    sites = [m.site(q) for q in range(n)]
    for q in range(n - 1):
        chi = sites[q].shape[2]
        X = np.eye(chi) + 0.4 * (rng.normal(size=(chi, chi)) + 1j * rng.normal(size=(chi, chi)))
        sites[q] = np.einsum("asb,bc->asc", sites[q], X)
        sites[q + 1] = np.einsum("cb,bsd->csd", np.linalg.inv(X), sites[q + 1])
    sites[0] = 1.7 * sites[0]
    g = O.OracleMPS(n, 256)
    g.set_state(sites, [m.lam(b) for b in range(n - 1)])
    psi = statevector(n, gates)
    u = np.random.default_rng(18).random((200, n))
    bits, logp = g.sample(u)
    ref_bits, ref_logp = sample_dense(psi, n, u)
    _assert_same_draws(bits, ref_bits, u, psi, n)
    assert np.array_equal(bits, ref_bits)
    assert np.max(np.abs(logp - ref_logp)) < 1e-9


def test_sampling_product_state_closed_form():
    """Ry(theta_q)|0> on every qubit: qubit q reads 0 with probability
    cos^2(theta_q / 2), independently of the others."""
    n = 10
    rng = np.random.default_rng(4)
    th = rng.uniform(0.2, 2.9, n)
    m = O.OracleMPS(n, 4)
    for q in range(n):
        m.apply((q, -1, W.ry(th[q])))
    u = rng.random((100, n))
    bits, logp = m.sample(u)
    p0 = np.cos(th / 2) ** 2
    assert np.array_equal(bits, (u >= p0[None, :]).astype(np.uint8))
    ref = np.where(bits == 0, np.log(p0)[None, :], np.log1p(-p0)[None, :]).sum(axis=1)
    assert np.max(np.abs(logp - ref)) < 1e-12


def test_sampling_ghz_closed_form():
    """GHZ: every string is all zeros or all ones with probability 1/2, and
    the first qubit drawn (n-1) decides which."""
    n = 16
    gates = [(0, -1, W.hadamard())] + [(j, j + 1, W.cnot()) for j in range(n - 1)]
    m = O.run_gates(n, 4, 0.0, gates)
    u = np.random.default_rng(6).random((64, n))
    bits, logp = m.sample(u)
    want = (u[:, n - 1] >= 0.5).astype(np.uint8)
    assert np.array_equal(bits, np.repeat(want[:, None], n, axis=1))
    assert np.max(np.abs(logp - math.log(0.5))) < 1e-13


def test_sampling_frequencies():
    """Frequencies of 20000 draws from a 5-qubit state against |psi|^2
    (total variation well inside the sampling noise of ~0.02)."""
    n = 5
    gates = nonlocal_circuit(n, 20, 7)
    m = O.run_gates(n, 64, 0.0, gates)
    u = np.random.default_rng(8).random((20000, n))
    bits, _ = m.sample(u)
    idx = bits.astype(np.int64) @ (1 << np.arange(n))
    freq = np.bincount(idx, minlength=2 ** n) / len(idx)
    prob = np.abs(statevector(n, gates)) ** 2
    assert 0.5 * np.abs(freq - prob).sum() < 0.03


# ---------------------------------------------------------------- canonical form (Sec. IV.A)

def _dense(sites):
    """Dense state of a chain of site tensors (index x = sum_q b_q 2^q),
    contracted here with numpy, independently of the oracle."""
    t = np.ones((1, 1), dtype=np.complex128)
    for a in sites:
        t = np.einsum("xa,asb->sxb", t, a).reshape(-1, a.shape[2])
    return t[:, 0]


def _generic_mps(n, dims, seed):
    """Sites of complex Gaussian entries: no canonical structure at all."""
    rng = np.random.default_rng(seed)
    sites = [(rng.standard_normal((dims[q], 2, dims[q + 1]))
              + 1j * rng.standard_normal((dims[q], 2, dims[q + 1]))) for q in range(n)]
    lams = [np.ones(dims[q + 1]) for q in range(n - 1)]
    return sites, lams


def _left_canonical_defect(m):
    worst = 0.0
    for q in range(m.n - 1):
        a = m.site(q).reshape(-1, m.site(q).shape[2])
        worst = max(worst, np.max(np.abs(a.conj().T @ a - np.eye(a.shape[1]))))
    return worst


def test_canonicalize_generic_gauge_against_brute_force():
    """Canonicalisation from a state with no structure (Gaussian sites, bond
    dimensions above the ranks the cuts allow): afterwards every site is
    left-canonical, the state equals the input divided by its norm, and
    lambda_b are the Schmidt values of that state at every cut (numpy SVD of
    the brute-force state vector); bond b keeps exactly its rank."""
    n = 9
    dims = [1, 3, 5, 9, 13, 13, 7, 4, 3, 1]
    sites, lams = _generic_mps(n, dims, 71)
    psi = _dense(sites)
    psi = psi / np.linalg.norm(psi)
    m = O.OracleMPS(n, 64)
    m.set_state(sites, lams)
    m.canonicalize()
    assert _left_canonical_defect(m) < 1e-12
    after = _dense([m.site(q) for q in range(n)])
    assert abs(np.linalg.norm(after) - 1.0) < 1e-12
    assert abs(abs(np.vdot(psi, after)) - 1.0) < 1e-12
    assert abs(np.vdot(psi, after) - 1.0) < 1e-12  # same state, same phase (no gate acted)
    for b in range(n - 1):
        ref = schmidt_values(psi, n, b)
        rank = int(np.sum(ref ** 2 > 1e-26))
        assert m.bond_dims()[b] == min(rank, 2 ** (b + 1), 2 ** (n - b - 1))
        assert np.max(np.abs(m.lam(b) - ref[: m.bond_dims()[b]])) < 1e-12


def test_canonicalize_leaves_a_canonical_state_unchanged():
    """On an exact canonical state (an untruncated circuit) the Schmidt
    values are already on the bonds: canonicalisation keeps them and the
    state."""
    cfg = W.config_small()
    m = O.OracleMPS(cfg.n, cfg.chi_max, cfg.cutoff)
    m.run_layers(cfg.layers)
    before = m.statevector()
    lam0 = [m.lam(b) for b in range(cfg.n - 1)]
    m.canonicalize()
    assert abs(abs(np.vdot(before, m.statevector())) - 1.0) < 1e-12
    for b in range(cfg.n - 1):
        assert np.max(np.abs(m.lam(b) - lam0[b])) < 1e-12


def test_canonicalize_truncation_is_the_optimal_cut():
    """Truncating canonicalisation with chi_max = 12 on an 8-qubit state whose
    only bond above 12 is the middle one (rank 16): the result is the best
    rank-12 approximation at that cut (Eckart-Young), so 1 - F equals the
    discarded weight sum_{j>12} sigma_j^2 of the exact state there, which is
    also what the statistics record; the other bonds keep their exact ranks."""
    n = 8
    layers = W.brickwork_haar(n, 8, 515)
    full = O.OracleMPS(n, 64)
    full.run_layers(layers)
    psi = full.statevector()
    sig = schmidt_values(psi, n, 3)
    assert int(np.sum(sig ** 2 > 1e-26)) == 16
    eps = float(np.sum(sig[12:] ** 2))
    m = O.OracleMPS(n, 12, 0.0)
    m.set_state([full.site(q) for q in range(n)], [full.lam(b) for b in range(n - 1)])
    m.canonicalize(truncate=True)
    assert list(m.bond_dims()) == [2, 4, 8, 12, 8, 4, 2]
    after = m.statevector()
    assert abs((1 - fidelity_dense(psi, after)) - eps) < 1e-12
    assert abs(m.stats()["sum_eps"] - eps) < 1e-12
    assert _left_canonical_defect(m) < 1e-12
    for b in range(n - 1):
        ref = schmidt_values(after, n, b)
        assert np.max(np.abs(m.lam(b) - ref[: m.bond_dims()[b]])) < 1e-12


# ---------------------------------------------------------------- bond propagation (Sec. III.A)

def _dense_gate(psi, n, q0, q1, g):
    """G on qubits (q0, q1) of a dense state (index x = sum_q b_q 2^q), rows of
    G in the basis |s_q0 s_q1> with s_q0 major."""
    t = psi.reshape([2] * n)  # axis k <-> qubit n-1-k
    a0, a1 = n - 1 - q0, n - 1 - q1
    t = np.moveaxis(t, (a0, a1), (0, 1)).reshape(4, -1)
    t = (np.asarray(g) @ t).reshape([2, 2] + [2] * (n - 2))
    return np.moveaxis(t, (0, 1), (a0, a1)).reshape(-1)


@pytest.mark.parametrize("gate", ["haar", "cnot"])
def test_propagation_matches_statevector(gate):
    """Gates on distant qubits by bond propagation, both orientations and
    distances 2 .. 7, without truncation: the brute-force state vector."""
    n = 8
    rng = np.random.default_rng(808)
    m = O.OracleMPS(n, 64)
    m.run_layers(W.brickwork_haar(n, 4, 809))
    psi = m.statevector()
    for (q0, q1) in [(0, 2), (5, 1), (1, 7), (7, 0), (3, 6), (6, 4)]:
        g = W.haar_u4(rng) if gate == "haar" else W.cnot()
        assert m.apply_2q_propagate(q0, q1, g) == O.OK
        psi = _dense_gate(psi, n, q0, q1, g)
        assert np.max(np.abs(m.statevector() - psi)) < 1e-12
    assert _left_canonical_defect(m) < 1e-12
    for b in range(n - 1):
        ref = schmidt_values(psi, n, b)
        assert np.max(np.abs(m.lam(b) - ref[: m.bond_dims()[b]])) < 1e-12


def test_propagation_ghz_and_operator_rank():
    """CNOTs from qubit 0 to every other qubit, in scrambled order, by bond
    propagation after H on qubit 0: GHZ with bond dimension 2 (Sec. V.A).  A
    product gate (operator rank 1) adds no entanglement; the identity leaves
    the state as it is."""
    n = 9
    m = O.OracleMPS(n, 16)
    m.apply((0, -1, W.hadamard()))
    for t in [5, 1, 8, 3, 2, 7, 4, 6]:
        assert m.apply_2q_propagate(0, t, W.cnot()) == O.OK
    psi = m.statevector()
    s2 = 1 / math.sqrt(2)
    assert abs(psi[0] - s2) < 1e-14 and abs(psi[-1] - s2) < 1e-14
    assert np.sum(np.abs(psi) > 1e-12) == 2
    assert list(m.bond_dims()) == [2] * (n - 1)
    before = m.statevector()
    assert m.apply_2q_propagate(1, 6, np.kron(W.rx(0.3), W.ry(1.1))) == O.OK
    assert list(m.bond_dims()) == [2] * (n - 1)
    assert m.apply_2q_propagate(7, 2, np.eye(4)) == O.OK
    assert np.max(np.abs(m.statevector() - _dense_gate(before, n, 1, 6, np.kron(W.rx(0.3), W.ry(1.1))))) < 1e-13


def test_propagation_truncation_is_a_right_to_left_schmidt_cut():
    """With chi_max below what the gate creates, the cuts happen from the
    right: the result equals the exact state G|psi> cut to its best rank
    chi_max at bond b-1, renormalised, then at b-2, ..., down to bond a
    (brute force, numpy SVD at each cut); the recorded discarded weight is
    the sum over the cuts, and each bond keeps the Schmidt values of its
    cut (a later cut further left changes the state, so for bonds right of
    bond a these are the values at the time of their own cut)."""
    n, chi = 9, 6
    rng = np.random.default_rng(909)
    src = O.OracleMPS(n, 64)
    src.run_layers(W.brickwork_haar(n, 3, 910))
    psi = src.statevector()
    m = O.OracleMPS(n, chi, 0.0)
    m.set_state([src.site(q) for q in range(n)], [src.lam(b) for b in range(n - 1)])
    q0, q1 = 2, 6
    g = W.haar_u4(rng)
    assert m.apply_2q_propagate(q0, q1, g) == O.OK
    phi = _dense_gate(psi, n, q0, q1, g)
    eps = 0.0
    kept = {}
    for b in range(q1 - 1, q0 - 1, -1):  # bonds b-1 .. a of the gate, right to left
        mat = phi.reshape(2 ** (n - b - 1), 2 ** (b + 1))
        u, s, vh = np.linalg.svd(mat, full_matrices=False)
        k = min(chi, int(np.sum(s ** 2 > (2 ** (n - b - 1)) * 2.0 ** -53 * s[0] ** 2)))
        eps += float(np.sum(s[k:] ** 2) / np.sum(s ** 2))
        kept[b] = s[:k] / np.linalg.norm(s[:k])
        phi = (u[:, :k] * s[:k]) @ vh[:k]
        phi = phi.reshape(-1) / np.linalg.norm(phi)
    got = m.statevector()
    assert 1 - fidelity_dense(phi, got) < 1e-12
    assert abs(m.stats()["sum_eps"] - eps) < 1e-12
    assert max(m.bond_dims()) <= chi
    assert list(m.bond_dims()[q0:q1]) == [len(kept[b]) for b in range(q0, q1)]
    for b in range(q0, q1):
        assert np.max(np.abs(m.lam(b) - kept[b])) < 1e-12
