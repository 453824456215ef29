"""Perfect sampling on the GPU (tnsim_sample) against the CPU oracle.

Parity is taken on one state: the GPU state is exported into an oracle
handle and both draw with the same uniforms.  Each bit is an integer decided
in float64 on both sides (u against the conditional probability), so the
strings must be identical; a mismatch could only come from a uniform within
rounding (~1e-14) of a conditional, which these seeds do not produce.  The
log-probabilities are sums of n float64 logs: compared at 1e-10.
"""
import math

import numpy as np
import pytest

from checkers import sample_dense, statevector
from gpu_helpers import dense_from_sites
from oracle import oracle as O
from paper_2601_04422_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2601_04422_amd import tnsim

    return tnsim


def _to_oracle(m):
    o = O.OracleMPS(m.n, 4096)
    o.set_state([m.site(q) for q in range(m.n)], [m.lam(b) for b in range(m.n - 1)])
    return o


def _draw(m, u):
    bits, logp = m.sample(u)
    return bits.cpu().numpy(), logp.cpu().numpy()


def _compare(bits, logp, rbits, rlogp, tol=1e-10):
    bad = np.nonzero((bits != rbits).any(axis=1))[0]
    assert bad.size == 0, f"shots {bad[:8]} differ from the oracle"
    assert np.max(np.abs(logp - rlogp)) < tol


@pytest.mark.parametrize("precision,storage", [("fp64", "c128"), ("bf16x6", "c64"),
                                               ("bf16x3", "c64"), ("f32acc", "c64")])
def test_sampling_vs_oracle(T, precision, storage):
    """A truncated random brickwork state (n=12, chi_max=32): 2000 shots."""
    n = 12
    m = T.MPS(n, 32, 1e-10, precision=precision, storage=storage)
    m.run_layers(W.brickwork_haar(n, 8, 41))
    assert max(m.bond_dims()) == 32
    u = np.random.default_rng(42).random((2000, n))
    bits, logp = _draw(m, u)
    rbits, rlogp = _to_oracle(m).sample(u)
    _compare(bits, logp, rbits, rlogp)
    assert len({tuple(b) for b in bits}) > 1000


def test_sampling_several_tiles_vs_oracle(T):
    """chi = 128 (two row tiles of the node GEMMs) and 700 shots (eleven
    column tiles, the last one ragged), on an imported left-canonical state."""
    n = 16
    dims = W.saturated_dims(n, 128)
    sites, lams = W.random_canonical_mps(n, dims, 77)
    m = T.MPS(n, 128)
    m.import_state(sites, lams)
    u = np.random.default_rng(43).random((700, n))
    bits, logp = _draw(m, u)
    rbits, rlogp = _to_oracle(m).sample(u)
    _compare(bits, logp, rbits, rlogp)


def test_sampling_non_canonical_gauge_vs_brute_force(T):
    """A state stored in a random non-orthonormal gauge and with norm != 1
    (imported): the draws equal sequential sampling from the brute-force
    state vector, so the left-block Gram matrices are used."""
    n = 8
    rng = np.random.default_rng(5)
    gates = [g for layer in W.brickwork_haar(n, 6, 12) for g in layer]
    o = O.run_gates(n, 256, 0.0, gates)
    sites = [o.site(q) for q in range(n)]
    for q in range(n - 1):
        chi = sites[q].shape[2]
        X = np.eye(chi) + 0.4 * (rng.normal(size=(chi, chi)) + 1j * rng.normal(size=(chi, chi)))
        sites[q] = np.einsum("asb,bc->asc", sites[q], X)
        sites[q + 1] = np.einsum("cb,bsd->csd", np.linalg.inv(X), sites[q + 1])
    sites[0] = 0.6 * sites[0]
    m = T.MPS(n, 256)
    m.import_state(sites, [o.lam(b) for b in range(n - 1)])
    psi = statevector(n, gates)
    assert np.max(np.abs(dense_from_sites(sites) / 0.6 - psi)) < 1e-10
    u = rng.random((500, n))
    bits, logp = _draw(m, u)
    rbits, rlogp = sample_dense(psi, n, u)
    _compare(bits, logp, rbits, rlogp, tol=1e-9)


def test_sampling_closed_forms(T):
    """GHZ on 60 qubits: every string is all zeros or all ones, decided by the
    first qubit drawn (n-1), probability 1/2 (two memo nodes per step).
    Ry(theta_q) product state on 40 qubits: qubit q reads 0 when
    u < cos^2(theta_q / 2)."""
    n = 60
    m = T.MPS(n, 8)
    m.run_gates(W.ghz(n))
    u = np.random.default_rng(7).random((4096, n))
    bits, logp = _draw(m, u)
    want = (u[:, n - 1] >= 0.5).astype(np.uint8)
    assert np.array_equal(bits, np.repeat(want[:, None], n, axis=1))
    assert np.max(np.abs(logp - math.log(0.5))) < 1e-12
    n = 40
    rng = np.random.default_rng(8)
    th = rng.uniform(0.2, 2.9, n)
    m = T.MPS(n, 4)
    m.apply_layer([(q, -1, W.ry(th[q])) for q in range(n)])
    u = rng.random((1000, n))
    bits, logp = _draw(m, u)
    p0 = np.cos(th / 2) ** 2
    assert np.array_equal(bits, (u >= p0[None, :]).astype(np.uint8))
    ref = np.where(bits == 0, np.log(p0)[None, :], np.log1p(-p0)[None, :]).sum(axis=1)
    assert np.max(np.abs(logp - ref)) < 1e-11


def test_sampling_in_chunks_equals_one_call(T):
    """Shots share partial contractions only within a call; splitting the
    shots over calls gives the same strings (and the workspace is reused)."""
    n = 14
    m = T.MPS(n, 64, 1e-12)
    m.run_layers(W.brickwork_haar(n, 10, 3))
    u = np.random.default_rng(9).random((900, n))
    bits, logp = _draw(m, u)
    b1, l1 = _draw(m, u[:300])
    b2, l2 = _draw(m, u[300:])
    assert np.array_equal(bits, np.concatenate([b1, b2]))
    assert np.max(np.abs(logp - np.concatenate([l1, l2]))) < 1e-12
    b3, l3 = _draw(m, u[:1])
    assert np.array_equal(b3, bits[:1])


def test_sampling_errors(T):
    import ctypes as C

    import torch

    n = 6
    m = T.MPS(n, 8)
    m.run_gates(W.ghz(n))
    bits, logp = m.sample(np.zeros((0, n)))
    assert bits.shape == (0, n)
    u = np.random.default_rng(1).random((10, n))
    u[4, 2] = 1.0
    with pytest.raises(T.TnsimError) as e:
        m.sample(u)
    assert e.value.code == T.E_ARG
    with pytest.raises(ValueError):
        m.sample(np.zeros((3, n + 1)))
    # a workspace sized for fewer shots than asked for
    lib = T.lib()
    ws_small = lib.tnsim_sample_workspace_bytes(C.byref(m.cfg), 4)
    ws_big = lib.tnsim_sample_workspace_bytes(C.byref(m.cfg), 10)
    assert 0 < ws_small < ws_big
    ws = torch.empty(ws_small, dtype=torch.uint8, device=m.device)
    ut = torch.as_tensor(np.random.default_rng(2).random((10, n)), device=m.device)
    b = torch.empty((10, n), dtype=torch.uint8, device=m.device)
    st = lib.tnsim_sample(m._h, C.c_void_p(ws.data_ptr()), ws_small, 10,
                          C.c_void_p(ut.data_ptr()), C.c_void_p(b.data_ptr()), None)
    assert st == T.E_CAPACITY
    # the handle still works after the errors
    bits, _ = m.sample(np.random.default_rng(3).random((5, n)))
    assert bits.shape == (5, n)


def test_sample_counts_histogram(T):
    """GHZ on 8 qubits: 3000 shots give only the two strings, in proportions
    within sampling noise of 1/2, and the counts add up to the shots."""
    n = 8
    m = T.MPS(n, 4)
    m.run_gates(W.ghz(n))
    counts = m.sample_counts(np.random.default_rng(11).random((3000, n)))
    assert set(counts) == {"0" * n, "1" * n}
    assert sum(counts.values()) == 3000
    assert abs(counts["0" * n] / 3000 - 0.5) < 0.04


def test_prepare_once_draw_many(T):
    """Weights built once serve several draws, each equal to a full sample;
    any change of the state makes a draw fail until prepared again."""
    n = 12
    m = T.MPS(n, 32, 1e-10)
    m.run_layers(W.brickwork_haar(n, 6, 77))
    m.sample_prepare(500)
    rng = np.random.default_rng(31)
    for shots in (500, 137, 1):
        u = rng.random((shots, n))
        b1, l1 = m.sample_draw(u)
        b2, l2 = m.sample(u)
        assert np.array_equal(b1.cpu().numpy(), b2.cpu().numpy())
        assert np.array_equal(l1.cpu().numpy(), l2.cpu().numpy())
    with pytest.raises(T.TnsimError) as e:
        m.sample_draw(rng.random((501, n)))
    assert e.value.code == T.E_CAPACITY
    m.apply_1q(3, W.rx(0.4))
    with pytest.raises(T.TnsimError) as e:
        m.sample_draw(rng.random((10, n)))
    assert e.value.code == T.E_ARG
    m.sample_prepare(10)
    u = rng.random((10, n))
    b1, _ = m.sample_draw(u)
    b2, _ = m.sample(u)
    assert np.array_equal(b1.cpu().numpy(), b2.cpu().numpy())
