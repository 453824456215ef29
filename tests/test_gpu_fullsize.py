"""Full-size parity: one batched layer at chi = 1024 (and chi = 256) from a
seeded synthetic left-canonical state, in the launch configuration the
benchmark times, checked against the CPU oracle on a sampled gate whose three
bonds are all at full size, and through invariants on every gate.

Sampled-gate comparison is gauge-free: the two-site product A_i' A_{i+1}'
(= U_k U_k^H theta' / N), the kept count k, the spectrum lambda_i' and the
discarded weight.  Tolerances: float64 path 1e-10 relative on the product and
spectrum; split-precision paths 1e-5 (float32-level operands, complex64
storage), well inside the 1e-6 state-fidelity requirement per gate.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_04422_amd import workloads as W

pytestmark = pytest.mark.gpu

N_SITES = 24


@pytest.fixture(scope="module")
def T():
    import torch

    assert torch.cuda.is_available()
    from paper_2601_04422_amd import tnsim

    return tnsim


def _state(chi, seed):
    dims = W.saturated_dims(N_SITES, chi)
    sites, lams = W.random_canonical_mps(N_SITES, dims, seed)
    return dims, sites, lams


def _layer(seed):
    """CNOTs dressed with seeded single-qubit rotations on the odd bonds."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(1, N_SITES - 1, 2):
        a, b, c, d = rng.uniform(0, 2 * np.pi, 4)
        u0 = W.rz(a) @ W.rx(b)
        u1 = W.rz(c) @ W.rx(d)
        out.append((j, j + 1, W.cnot() @ np.kron(u0, u1)))
    return out


def _block(a, b):
    return np.einsum("asb,btc->astc", a, b).reshape(a.shape[0] * 2, 2 * b.shape[2])


@pytest.mark.parametrize("chi,precision,storage,tol", [
    (1024, "bf16x6", "c64", 1e-5),
    (1024, "fp64", "c128", 1e-10),
    (256, "f32acc", "c64", 1e-5),
])
def test_full_size_layer_vs_oracle(T, chi, precision, storage, tol):
    dims, sites, lams = _state(chi, 1000 + chi)
    layer = _layer(7)
    m = T.MPS(N_SITES, chi, 1e-12, precision=precision, storage=storage)
    m.import_state(sites, lams)
    assert m.apply_layer(layer) == T.OK
    # invariants on every gate of the layer
    for (i, _, _) in layer:
        a = m.site(i).reshape(-1, m.bond_dims()[i])
        gram = a.conj().T @ a
        assert np.max(np.abs(gram - np.eye(gram.shape[0]))) < (1e-10 if storage == "c128" else 1e-5)
        assert abs(np.sum(m.lam(i) ** 2) - 1) < 1e-10
    # sampled gate with chiL = chiM = chiR = chi, against the oracle
    i = N_SITES // 2 - 1
    assert dims[i] == dims[i + 1] == dims[i + 2] == chi
    g = [x for x in layer if x[0] == i][0][2]
    O.set_threads(16)
    o = O.OracleMPS(N_SITES, chi, 1e-12)
    o.set_state(sites, lams)
    assert o.apply_2q(i, i + 1, g) == O.OK
    st = o.stats()
    assert m.bond_dims()[i] == o.bond_dims()[i] == st["last_k"]
    lam_g, lam_o = m.lam(i), o.lam(i)
    assert np.max(np.abs(lam_g - lam_o)) / lam_o[0] < tol
    pg = _block(m.site(i), m.site(i + 1))
    po = _block(o.site(i), o.site(i + 1))
    assert np.linalg.norm(pg - po) / np.linalg.norm(po) < tol
    assert st["last_eps"] > 0


def test_gate_beyond_qr_rows_vs_oracle(T):
    """chi = 1100: M is 2200 x 2200, more rows than one QR panel workgroup
    holds, so even the mixed path takes the plain Jacobi on M.  One gate
    against the oracle (k, spectrum, two-site product)."""
    chi, tol = 1100, 1e-5
    dims, sites, lams = _state(chi, 77)
    i = N_SITES // 2 - 1
    assert dims[i] == dims[i + 1] == dims[i + 2] == chi
    g = W.cnot() @ np.kron(W.rz(0.4) @ W.rx(1.2), W.rz(2.2) @ W.rx(0.3))
    m = T.MPS(N_SITES, chi, 1e-12, precision="bf16x6", storage="c64")
    m.import_state(sites, lams)
    assert m.apply_2q(i, i + 1, g) == T.OK
    O.set_threads(16)
    o = O.OracleMPS(N_SITES, chi, 1e-12)
    o.set_state(sites, lams)
    assert o.apply_2q(i, i + 1, g) == O.OK
    assert m.bond_dims()[i] == o.bond_dims()[i]
    lam_g, lam_o = m.lam(i), o.lam(i)
    assert np.max(np.abs(lam_g - lam_o)) / lam_o[0] < tol
    pg = _block(m.site(i), m.site(i + 1))
    po = _block(o.site(i), o.site(i + 1))
    assert np.linalg.norm(pg - po) / np.linalg.norm(po) < tol


def test_sampling_full_size_vs_oracle_amplitudes(T):
    """Perfect sampling at chi = 1024 (n = 24, the middle bonds at 1024,
    complex128 sites) with 1000 shots (a ragged last column tile): every drawn
    string's log-probability equals log |<x|psi>|^2 from the oracle's
    amplitude contraction of the same state (norm 1 to rounding: the sites
    are float64 isometries), and the strings are those of the same draw split
    over two calls."""
    import math

    dims, sites, lams = _state(1024, 2031)
    m = T.MPS(N_SITES, 1024)
    m.import_state(sites, lams)
    o = O.OracleMPS(N_SITES, 1024)
    o.set_state([m.site(q) for q in range(N_SITES)], [m.lam(b) for b in range(N_SITES - 1)])
    u = np.random.default_rng(2032).random((1000, N_SITES))
    bits, logp = m.sample(u)
    bits, logp = bits.cpu().numpy(), logp.cpu().numpy()
    assert len({tuple(b) for b in bits}) == 1000
    for i in range(0, 1000, 37):
        ref = math.log(abs(o.amplitude(bits[i])) ** 2)
        assert abs(logp[i] - ref) < 1e-9, (i, logp[i], ref)
    b2, l2 = m.sample(u[500:])
    assert np.array_equal(b2.cpu().numpy(), bits[500:])
    assert np.max(np.abs(l2.cpu().numpy() - logp[500:])) < 1e-12


def test_two_layers_flat_spectrum_chi1024(T):
    """Two consecutive chi = 1024 layers in the benchmark's batched form
    (float64, complex128 sites, QR-preconditioned Jacobi, one stream of its
    own so the sweeps replay as a graph) on a state whose Schmidt spectra are
    random-circuit-like (quarter-circle law: flat, no gap at the cut).
    Layer 1 acts on the odd bonds, layer 2 on the even bonds.  Checked
    against the oracle (float64 bound 1e-10):
      * layer 1, gates (i-1, i) and (i+1, i+2) from the input state: k, the
        spectrum and the two-site product (whose outer bonds keep the input's
        basis, so the product is gauge-free);
      * layer 2, gate (i, i+1), which reads both of those gates' outputs: the
        oracle applies it to the GPU's state after layer 1 (so bonds i-1 and
        i+1 carry the same basis on both sides): k, spectrum, discarded
        weight and two-site product."""
    import torch

    chi, tol = 1024, 1e-10
    dims = W.saturated_dims(N_SITES, chi)
    sites, lams = W.random_canonical_mps(N_SITES, dims, 3301, profile="flat")
    rng = np.random.default_rng(3302)

    def dressed():
        a, b, c, d = rng.uniform(0, 2 * np.pi, 4)
        return W.cnot() @ np.kron(W.rz(a) @ W.rx(b), W.rz(c) @ W.rx(d))

    l1 = [(j, j + 1, dressed()) for j in range(1, N_SITES - 1, 2)]
    l2 = [(j, j + 1, dressed()) for j in range(2, N_SITES - 1, 2)]
    i = N_SITES // 2
    assert i % 2 == 0 and dims[i - 1] == dims[i] == dims[i + 1] == dims[i + 2] == chi
    m = T.MPS(N_SITES, chi, 1e-12, precision="fp64", storage="c128", svd_precondition=True,
              stream=torch.cuda.Stream())
    m.import_state(sites, lams)
    assert m.apply_layer(l1) == T.OK
    after1 = ([m.site(q) for q in range(N_SITES)], [m.lam(b) for b in range(N_SITES - 1)])
    assert m.apply_layer(l2) == T.OK
    # the left site of every layer-2 gate is U_k (isometric); the left sites
    # of the layer-1 gates became right sites of layer-2 gates, which a cut
    # leaves only approximately left-canonical
    for (j, _, _) in l2:
        a = m.site(j).reshape(-1, m.bond_dims()[j])
        gram = a.conj().T @ a
        assert np.max(np.abs(gram - np.eye(gram.shape[0]))) < 1e-10
    for (j, _, _) in l1 + l2:
        assert abs(np.sum(m.lam(j) ** 2) - 1) < 1e-10
    O.set_threads(16)

    def check(o, j, gs, gl, eps_min):
        st = o.stats()
        assert st["last_eps"] > eps_min  # a real cut on a flat spectrum
        assert len(gl[j]) == o.bond_dims()[j] == st["last_k"]
        assert np.max(np.abs(gl[j] - o.lam(j))) / o.lam(j)[0] < tol
        pg = _block(gs[j], gs[j + 1])
        po = _block(o.site(j), o.site(j + 1))
        assert np.linalg.norm(pg - po) / np.linalg.norm(po) < tol

    o = O.OracleMPS(N_SITES, chi, 1e-12)
    o.set_state(sites, lams)
    for (j, jj, g) in l1:
        if j in (i - 1, i + 1):
            assert o.apply_2q(j, jj, g) == O.OK
            # (i+1, i+2) has chi_R = 512: M is 2048 x 1024 and chi_max does not cut
            check(o, j, after1[0], after1[1], 1e-4 if j == i - 1 else -1.0)
    o = O.OracleMPS(N_SITES, chi, 1e-12)
    o.set_state(*after1)
    g2 = [x for x in l2 if x[0] == i][0][2]
    assert o.apply_2q(i, i + 1, g2) == O.OK
    check(o, i, [m.site(q) for q in range(N_SITES)], [m.lam(b) for b in range(N_SITES - 1)],
          1e-4)
    assert m.bond_dims()[i] == chi
