"""GPU path against the CPU oracle (and the brute-force state vector).

Tolerances: the float64 path is compared at 1e-12 on amplitudes when no
truncation happens, and at 1e-10 on Schmidt spectra and 1 - F when it does
(both sides take the same truncation decisions on generic random inputs).
"""
import math

import numpy as np
import pytest

from checkers import amplitude_index, fidelity_dense, statevector
from gpu_helpers import gpu_statevector, mps_fidelity_gpu_vs_oracle
from oracle import oracle as O
from paper_2601_04422_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2601_04422_amd import tnsim

    return tnsim


def _oracle_fid(g, o):
    return mps_fidelity_gpu_vs_oracle(g, o, lambda n: O.OracleMPS(n, 4096))


@pytest.mark.parametrize("mode", ["layer", "per_gate"])
def test_small_brickwork_amplitudes(T, mode):
    cfg = W.config_small()
    m = T.MPS(cfg.n, cfg.chi_max, cfg.cutoff)
    if mode == "layer":
        m.run_layers(cfg.layers)
    else:
        m.run_gates(cfg.gates())
    ref = statevector(cfg.n, cfg.gates())
    got = gpu_statevector(m)
    assert np.max(np.abs(got - ref)) < 1e-12
    rng = np.random.default_rng(3)
    for _ in range(8):
        bits = rng.integers(0, 2, cfg.n)
        assert abs(m.amplitude(bits) - ref[amplitude_index(bits)]) < 1e-12
    o = O.OracleMPS(cfg.n, cfg.chi_max, cfg.cutoff)
    o.run_layers(cfg.layers)
    assert list(m.bond_dims()) == list(o.bond_dims())
    for b in range(cfg.n - 1):
        assert np.max(np.abs(m.lam(b) - o.lam(b))) < 1e-12


def test_ghz_n100(T):
    n = 100
    m = T.MPS(n, 64)
    m.run_gates(W.ghz(n))
    assert abs(m.amplitude([0] * n) - 1 / math.sqrt(2)) < 1e-14
    assert abs(m.amplitude([1] * n) - 1 / math.sqrt(2)) < 1e-14
    assert max(m.bond_dims()) == 2


def test_product_state_closed_forms(T):
    n = 6
    m = T.MPS(n, 4)
    th, ph, al = [0.3, 1.7, 3.0], [1.1, -0.4, 2.5], [2.0, 0.5, 4.4]
    layer1 = [(2 * r, -1, W.ry(th[r])) for r in range(3)] + \
             [(2 * r + 1, -1, W.rx(al[r])) for r in range(3)]
    layer2 = [(2 * r, -1, W.rz(ph[r])) for r in range(3)]
    m.run_layers([layer1, layer2])

    def e(q, c):
        s = ["I"] * n
        s[q] = c
        return m.expect("".join(s))

    for r in range(3):
        assert abs(e(2 * r, "Z") - math.cos(th[r])) < 1e-14
        assert abs(e(2 * r, "X") - math.sin(th[r]) * math.cos(ph[r])) < 1e-14
        assert abs(e(2 * r, "Y") - math.sin(th[r]) * math.sin(ph[r])) < 1e-14
        assert abs(e(2 * r + 1, "Z") - math.cos(al[r])) < 1e-14
        assert abs(e(2 * r + 1, "Y") + math.sin(al[r])) < 1e-14


@pytest.mark.parametrize("seed", [11, 12])
def test_mixed_gates_reversed_orientation(T, seed):
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
    m = T.MPS(n, 64)
    m.run_gates(gates)
    ref = statevector(n, gates)
    assert np.max(np.abs(gpu_statevector(m) - ref)) < 1e-12


@pytest.mark.parametrize("n,depth,chi,cutoff", [(16, 12, 12, 1e-10), (18, 14, 100, 1e-10),
                                                (12, 10, 5, 0.0)])
def test_truncating_brickwork_vs_oracle(T, n, depth, chi, cutoff):
    """Truncation active; chi_max values that leave ragged tiles."""
    layers = W.brickwork_haar(n, depth, 900 + n)
    m = T.MPS(n, chi, cutoff)
    m.run_layers(layers)
    o = O.OracleMPS(n, chi, cutoff)
    o.run_layers(layers)
    assert list(m.bond_dims()) == list(o.bond_dims())
    for b in range(n - 1):
        assert np.max(np.abs(m.lam(b) - o.lam(b))) < 1e-10
    st_g, st_o = m.stats(), o.stats()
    assert abs(st_g["sum_eps"] - st_o["sum_eps"]) <= 1e-10 * max(1.0, st_o["sum_eps"])
    assert 1 - _oracle_fid(m, o) < 1e-10


def test_layer_permutation_bit_exact(T):
    n = 14
    layers = W.brickwork_haar(n, 8, 31)
    a = T.MPS(n, 16, 1e-10)
    b = T.MPS(n, 16, 1e-10)
    rng = np.random.default_rng(0)
    for layer in layers:
        assert a.apply_layer(layer) == T.OK
        perm = rng.permutation(len(layer))
        assert b.apply_layer([layer[i] for i in perm]) == T.OK
    for q in range(n):
        assert np.array_equal(a.site(q), b.site(q))
    assert a.stats()["sum_eps"] > 0


def test_expectations_and_overlap_vs_oracle(T):
    n = 12
    layers = W.brickwork_haar(n, 8, 5)
    m = T.MPS(n, 32, 0.0)
    m.run_layers(layers)
    o = O.OracleMPS(n, 32, 0.0)
    o.run_layers(layers)
    rng = np.random.default_rng(8)
    for _ in range(6):
        p = "".join(rng.choice(list("IXYZ"), n))
        assert abs(m.expect(p) - o.expect(p)) < 1e-12
    assert abs(m.norm2() - 1) < 1e-12
    m2 = T.MPS(n, 32, 0.0)
    m2.run_layers(layers[:-1])
    o2 = O.OracleMPS(n, 32, 0.0)
    o2.run_layers(layers[:-1])
    assert abs(m.overlap(m2) - o.overlap(o2)) < 1e-12


def test_import_export_roundtrip_and_copy(T):
    n = 10
    dims = W.saturated_dims(n, 8)
    sites, lams = W.random_canonical_mps(n, dims, 4)
    m = T.MPS(n, 8)
    m.import_state(sites, lams)
    for q in range(n):
        assert np.array_equal(m.site(q), sites[q])
    c = T.MPS(n, 8, storage="c64")
    c.copy_from(m)
    for q in range(n):
        assert np.max(np.abs(c.site(q) - sites[q])) < 1e-6
    assert abs(abs(m.overlap(c)) - 1) < 1e-6


def test_errors_leave_state_unchanged(T):
    n = 6
    m = T.MPS(n, 8)
    g = W.cnot()
    assert m.apply_layer([(0, 1, g), (1, 2, g)]) == T.E_OVERLAP
    assert m.apply_layer([(0, 2, g)]) == T.E_NONLOCAL
    assert m.apply_layer([(5, 6, g)]) == T.E_ARG
    assert m.apply_2q(0, 6, g) == T.E_ARG
    bad = np.array(g, dtype=np.complex128)
    bad[1, 1] = np.nan
    assert m.apply_2q(0, 1, bad) == T.E_ARG
    assert m.apply_2q(0, 3, bad) == T.E_ARG
    assert m.apply_layer([(2, 3, bad)]) == T.E_ARG
    assert m.apply_circuit([(1, 4, bad)]) == T.E_ARG
    with pytest.raises(T.TnsimError):
        m.apply_1q(0, np.array([[1, 0], [0, np.inf]]))
    assert list(m.bond_dims()) == [1] * (n - 1)
    assert abs(m.amplitude([0] * n) - 1) < 1e-15
    nc = T.MPS(n, 8, jacobi_max_sweeps=1)
    rng = np.random.default_rng(2)
    assert nc.apply_2q(2, 3, W.haar_u4(rng)) == T.E_NOCONV
    assert list(nc.bond_dims()) == [1] * (n - 1)
    # the handle stays usable after NOCONV
    assert abs(nc.amplitude([0] * n) - 1) < 1e-15


# ---------------------------------------------------------------- mixed precision paths

@pytest.mark.parametrize("precision,bound", [("f32acc", 1e-9), ("bf16x6", 1e-9), ("bf16x3", 1e-7)])
def test_mixed_precision_vs_oracle(T, precision, bound):
    """Complex64 storage with the matrix-core contraction / write-back against
    the float64 oracle.  Tolerance: state fidelity error <= 1e-6 (the
    requirement), with the bound expected from the arithmetic (float32-level
    operands, ~1e-7 relative per gate for f32acc/bf16x6, ~2^-16 for bf16x3)."""
    n, depth, chi = 16, 12, 24
    layers = W.brickwork_haar(n, depth, 4242)
    m = T.MPS(n, chi, 1e-10, precision=precision, storage="c64")
    m.run_layers(layers)
    o = O.OracleMPS(n, chi, 1e-10)
    o.run_layers(layers)
    err = 1 - _oracle_fid(m, o)
    assert err <= 1e-6
    assert err <= bound, err
    for q in (0, 7, 15):
        s = ["I"] * n
        s[q] = "Z"
        assert abs(m.expect("".join(s)) - o.expect("".join(s))) < 1e-5


def test_mixed_untruncated_amplitudes(T):
    cfg = W.config_small()
    m = T.MPS(cfg.n, cfg.chi_max, cfg.cutoff, precision="bf16x6", storage="c64")
    m.run_layers(cfg.layers)
    ref = statevector(cfg.n, cfg.gates())
    got = gpu_statevector(m)
    assert np.max(np.abs(got - ref)) < 1e-6
    assert 1 - fidelity_dense(got, ref) < 1e-10


# ---------------------------------------------------------------- several circuits, one batch

def test_multi_circuit_batch_vs_oracle(T):
    """Independent circuits of uneven n, depth and chi_max advanced layer by
    layer with all their two-qubit gates in shared launches."""
    specs = [(9, 6, 4, 11), (14, 9, 16, 12), (6, 7, 8, 13), (20, 5, 32, 14), (11, 8, 100, 15)]
    ms, circuits = [], []
    for k, (n, depth, chi, seed) in enumerate(specs):
        ms.append(T.MPS(n, chi, 1e-10, max_layer_gates=(64 if k == 0 else 3)))
        circuits.append(W.brickwork_haar(n, depth, seed))
    depth_max = max(len(c) for c in circuits)
    for l in range(depth_max):
        active = [k for k in range(len(ms)) if l < len(circuits[k])]
        st = T.apply_layer_multi([ms[k] for k in active], [circuits[k][l] for k in active])
        assert st == T.OK
    for k, (n, depth, chi, seed) in enumerate(specs):
        o = O.OracleMPS(n, chi, 1e-10)
        o.run_layers(circuits[k])
        assert list(ms[k].bond_dims()) == list(o.bond_dims())
        assert 1 - _oracle_fid(ms[k], o) < 1e-10
        for b in range(n - 1):
            assert np.max(np.abs(ms[k].lam(b) - o.lam(b))) < 1e-10


@pytest.mark.parametrize("precision,storage", [("fp64", "c128"), ("bf16x6", "c64")])
def test_graph_replay_matches_eager(T, precision, storage):
    """A non-default stream captures each batch's Jacobi sweep as a HIP graph
    and replays it once per sweep (with the host's convergence check and
    other eager work between replays); every result must equal the eager
    launches bit for bit (float64 plain Jacobi, and the mixed path with the
    QR-preconditioned SVD)."""
    import torch

    n = 16
    layers = W.brickwork_haar(n, 10, 77)
    s = torch.cuda.Stream()
    g = T.MPS(n, 24, 1e-10, precision=precision, storage=storage, stream=s)
    e = T.MPS(n, 24, 1e-10, precision=precision, storage=storage)
    for layer in layers:
        assert g.apply_layer(layer) == T.OK
        assert e.apply_layer(layer) == T.OK
        assert g.stats()["last_sweeps"] >= 2
    for q in range(n):
        assert np.array_equal(g.site(q), e.site(q))
    for b in range(n - 1):
        assert np.array_equal(g.lam(b), e.lam(b))


# ---------------------------------------------------------------- QR-preconditioned SVD

@pytest.mark.parametrize("n,depth,chi,cutoff", [(16, 12, 12, 1e-10), (18, 14, 100, 1e-10),
                                                (12, 10, 5, 0.0), (14, 12, 64, 0.0)])
def test_qr_preconditioned_vs_oracle(T, n, depth, chi, cutoff):
    """float64 arithmetic with the QR-preconditioned Jacobi (square and tall M
    take it, wide M the plain path): same bond dimensions, spectra and
    discarded weight as the oracle's plain Jacobi, at the float64 tolerances."""
    layers = W.brickwork_haar(n, depth, 700 + n + chi)
    m = T.MPS(n, chi, cutoff, svd_precondition=True)
    m.run_layers(layers)
    o = O.OracleMPS(n, chi, cutoff)
    o.run_layers(layers)
    assert list(m.bond_dims()) == list(o.bond_dims())
    for b in range(n - 1):
        assert np.max(np.abs(m.lam(b) - o.lam(b))) < 1e-10
    st_g, st_o = m.stats(), o.stats()
    assert abs(st_g["sum_eps"] - st_o["sum_eps"]) <= 1e-10 * max(1.0, st_o["sum_eps"])
    assert 1 - _oracle_fid(m, o) < 1e-10
    for (q0, q1, _) in layers[-1]:  # the left site of each last gate is U_k, an isometry
        a = m.site(min(q0, q1))
        a = a.reshape(-1, a.shape[2])
        assert np.max(np.abs(a.conj().T @ a - np.eye(a.shape[1]))) < 1e-11


def test_qr_preconditioned_amplitudes(T):
    cfg = W.config_small()
    m = T.MPS(cfg.n, cfg.chi_max, cfg.cutoff, svd_precondition=True)
    m.run_layers(cfg.layers)
    ref = statevector(cfg.n, cfg.gates())
    assert np.max(np.abs(gpu_statevector(m) - ref)) < 1e-12
    g = T.MPS(9, 16, svd_precondition=True)
    rng = np.random.default_rng(21)
    gates = []
    for _ in range(30):
        j = int(rng.integers(0, 8))
        gates.append((j, j + 1, W.haar_u4(rng)) if rng.random() < 0.5 else (j + 1, j, W.haar_u4(rng)))
    g.run_gates(gates)
    assert np.max(np.abs(gpu_statevector(g) - statevector(9, gates))) < 1e-12


def test_fp64_rate_probe(T):
    """The float64 rate probe runs each form and reports a rate in a sane
    range (above 1 TFLOP/s, below twice the published 78.6); a unit outside
    the four is rejected."""
    m = T.MPS(4, 2)
    for unit in ("mfma", "valu", "mixed", "mfma4"):
        r = m.probe_fp64(unit, 200)
        assert 1.0 < r < 2 * 78.6, (unit, r)
    assert T.lib().tnsim_probe_fp64(m._h, 4, 10, T.C.byref(T.C.c_double())) == T.E_ARG


def test_autotuned_launch_shapes(T):
    """The rows per rotation workgroup never change a result: a handle with
    the tuned rotation shapes (and the built-in Gram K-split) gives the same
    state bit for bit as one on the built-in rules.  The tuned Gram K-split
    only reorders the Gram's row sums: the full tuned table agrees to
    rounding (same bond dimensions, Schmidt values to 1e-12)."""
    n = 16
    layers = W.brickwork_haar(n, 10, 55)
    a = T.MPS(n, 24, 1e-10, precision="bf16x6", storage="c64")
    b = T.MPS(n, 24, 1e-10, precision="bf16x6", storage="c64")
    table = a.autotune()
    assert len(table) == 8
    assert all(t in (64, 128, 256, 512) for t in table[:4])
    assert all(k in (1, 2, 4, 8, 16) for k in table[4:])
    a.set_autotune(table[:4] + [0, 0, 0, 0])
    a.run_layers(layers)
    b.run_layers(layers)
    for q in range(n):
        assert np.array_equal(a.site(q), b.site(q))
    for k in range(n - 1):
        assert np.array_equal(a.lam(k), b.lam(k))
    c = T.MPS(n, 24, 1e-10)
    d = T.MPS(n, 24, 1e-10)
    c.set_autotune(table)
    c.run_layers(layers)
    d.run_layers(layers)
    assert list(c.bond_dims()) == list(d.bond_dims())
    for k in range(n - 1):
        assert np.max(np.abs(c.lam(k) - d.lam(k))) < 1e-12
    with pytest.raises(Exception):
        c.set_autotune(table[:4] + [3, 0, 0, 0])


# ---------------------------------------------------------------- circuit scheduler

@pytest.mark.parametrize("precision,storage,tol,ltol", [("fp64", "c128", 1e-10, 1e-10),
                                                        ("bf16x6", "c64", 1e-9, 1e-6)])
def test_circuit_scheduler_vs_oracle(T, precision, storage, tol, ltol):
    """The whole circuit in one call (gates of consecutive layers overlap)
    against the oracle applying it gate by gate: same bond dimensions and
    spectra, fidelity at the path's tolerance."""
    n, depth, chi = 18, 14, 40
    layers = W.brickwork_haar(n, depth, 4321)
    gates = [g for layer in layers for g in layer]
    m = T.MPS(n, chi, 1e-10, precision=precision, storage=storage)
    m.run_circuit(gates)
    o = O.OracleMPS(n, chi, 1e-10)
    o.run_layers(layers)
    assert list(m.bond_dims()) == list(o.bond_dims())
    for b in range(n - 1):
        assert np.max(np.abs(m.lam(b) - o.lam(b))) < ltol
    assert 1 - _oracle_fid(m, o) < tol
    lb = m.last_batch()
    assert len(lb) == sum(1 for g in gates if g[1] >= 0)


def test_circuit_scheduler_mixed_gates_amplitudes(T):
    """Interleaved one- and two-qubit gates on shared qubits, both
    orientations, without truncation: amplitudes against brute force."""
    rng = np.random.default_rng(99)
    n = 9
    gates = []
    for _ in range(60):
        if rng.random() < 0.35:
            q = int(rng.integers(0, n))
            gates.append((q, -1, W.rot("XYZ"[int(rng.integers(0, 3))], rng.uniform(0, 6.3))))
        else:
            j = int(rng.integers(0, n - 1))
            g = W.haar_u4(rng)
            gates.append((j, j + 1, g) if rng.random() < 0.5 else (j + 1, j, g))
    m = T.MPS(n, 64)
    m.run_circuit(gates)
    assert np.max(np.abs(gpu_statevector(m) - statevector(n, gates))) < 1e-12
    c = T.MPS(n, 64)
    assert c.apply_circuit([(0, n, W.cnot())]) == T.E_ARG


@pytest.mark.parametrize("precision,storage", [("fp64", "c128"), ("bf16x6", "c64")])
def test_degenerate_sizes_vs_oracle(T, precision, storage):
    """Smallest shapes: two qubits, and chi_max = 1 (every two-qubit gate
    truncates to one Schmidt value), on the plain and the preconditioned SVD."""
    tol = 1e-12 if storage == "c128" else 1e-6
    rng = np.random.default_rng(17)
    gates = [(0, 1, W.haar_u4(rng)), (1, 0, W.haar_u4(rng)), (0, -1, W.rot("Y", 0.7))]
    m = T.MPS(2, 2, precision=precision, storage=storage)
    m.run_gates(gates)
    assert np.max(np.abs(gpu_statevector(m) - statevector(2, gates))) < tol
    layers = W.brickwork_haar(8, 6, 23)
    g = T.MPS(8, 1, 0.0, precision=precision, storage=storage)
    g.run_layers(layers)
    o = O.OracleMPS(8, 1, 0.0)
    o.run_layers(layers)
    assert list(g.bond_dims()) == [1] * 7
    # complex64 sites carry about 6e-8 relative rounding into the weights
    assert abs(g.stats()["sum_eps"] - o.stats()["sum_eps"]) < (1e-9 if storage == "c128" else 1e-6)
    assert 1 - _oracle_fid(g, o) < (1e-10 if storage == "c128" else 1e-6)


# ---------------------------------------------------------------- non-local gates

@pytest.mark.parametrize("mode", ["per_gate", "circuit"])
@pytest.mark.parametrize("precision,storage,tol", [("fp64", "c128", 1e-12), ("bf16x6", "c64", 1e-6)])
def test_nonlocal_gates_vs_statevector(T, mode, precision, storage, tol):
    """Gates on distant qubits (SWAP chains, Sec. IV.A), one call per gate and
    as one scheduled circuit, without truncation: amplitudes against brute force."""
    from test_oracle_pins import nonlocal_circuit

    n = 7
    gates = nonlocal_circuit(n, 30, 314)
    m = T.MPS(n, 256, precision=precision, storage=storage)
    if mode == "per_gate":
        m.run_gates(gates)
    else:
        m.run_circuit(gates)
    assert np.max(np.abs(gpu_statevector(m) - statevector(n, gates))) < tol


def test_nonlocal_truncating_vs_oracle(T):
    """Distant gates with truncation: every SWAP is a truncated gate, so the
    GPU must take the oracle's SWAP chain to match it."""
    from test_oracle_pins import nonlocal_circuit

    n, chi = 14, 16
    gates = nonlocal_circuit(n, 50, 2718)
    m = T.MPS(n, chi, 1e-10)
    m.run_circuit(gates)
    o = O.OracleMPS(n, chi, 1e-10)
    o.run(gates)
    assert list(m.bond_dims()) == list(o.bond_dims())
    for b in range(n - 1):
        assert np.max(np.abs(m.lam(b) - o.lam(b))) < 1e-10
    assert 1 - _oracle_fid(m, o) < 1e-10
    assert abs(m.stats()["sum_eps"] - o.stats()["sum_eps"]) < 1e-10
