"""Adjoint gradients on the GPU against closed forms, the oracle's parameter
shift (exact without truncation) and central finite differences of the GPU
forward (binding check with truncation).

Tolerance: 1e-4 relative (L2 norm of the error over the L2 norm of the
reference), the requirement for gradients; the untruncated comparison with
parameter shift is held to 1e-8."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_04422_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch

    assert torch.cuda.is_available()
    from paper_2601_04422_amd import tnsim

    return tnsim


def _spec(n, nl, ladder=True):
    qs, ps, axes = W.ansatz_structure(n, nl, ladder)
    gates = [(q0, q1, W.cnot() if q1 >= 0 else np.eye(2)) for (q0, q1) in qs]
    n_params = 2 * n * nl
    rot_axis = np.zeros(n_params, dtype=np.int32)
    for p, ax in zip(ps, axes):
        if p >= 0:
            rot_axis[p] = ax
    per_layer = 2 * n + (n - 1 if ladder else 0)
    seg = [l * per_layer for l in range(nl)]
    paulis = W.zz_chain(n)
    return gates, ps, rot_axis, seg, paulis, [1.0] * len(paulis)


def _loss_gpu(T, n, chi, angles, spec):
    gates, ps, ax, seg, paulis, coeffs = spec
    m = T.MPS(n, chi, 0.0)
    return m.forward_checkpointed(gates, ps, ax, angles, seg, paulis, coeffs)


def test_closed_form_without_cnots(T):
    n = 6
    angles = W.ansatz_angles(n, 1, 42)
    spec = _spec(n, 1, ladder=False)
    m = T.MPS(n, 8, 0.0)
    loss = m.forward_checkpointed(*spec[:2], spec[2], angles, *spec[3:])
    th = angles[0::2]
    assert abs(loss - sum(math.cos(th[i]) * math.cos(th[i + 1]) for i in range(n - 1))) < 1e-13
    g = m.backward(1.0)
    ref = np.zeros_like(angles)
    for i in range(n):
        nb = (math.cos(th[i - 1]) if i > 0 else 0.0) + (math.cos(th[i + 1]) if i < n - 1 else 0.0)
        ref[2 * i] = -math.sin(th[i]) * nb
    assert np.max(np.abs(g - ref)) < 1e-12


@pytest.mark.parametrize("n,nl", [(5, 2), (8, 3)])
def test_untruncated_vs_oracle_parameter_shift(T, n, nl):
    angles = W.ansatz_angles(n, nl, 7 + n)
    spec = _spec(n, nl)
    m = T.MPS(n, 64, 0.0)
    loss = m.forward_checkpointed(spec[0], spec[1], spec[2], angles, *spec[3:])
    g = m.backward(1.0)
    make = lambda a: W.ansatz_gates(a, n, nl)
    o = O.run_gates(n, 64, 0.0, make(angles))
    assert abs(loss - O.loss_pauli_sum(o, spec[4], spec[5])) < 1e-12
    ref = O.parameter_shift(make, angles, n, 64, 0.0, spec[4], spec[5])
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-8


def test_truncated_vs_finite_differences(T):
    """chi_max small enough that the later CNOTs truncate: the adjoint must
    match central differences (h = 1e-4) of the same truncated forward."""
    n, nl, chi = 10, 4, 6
    angles = W.ansatz_angles(n, nl, 99)
    spec = _spec(n, nl)
    m = T.MPS(n, chi, 0.0)
    m.forward_checkpointed(spec[0], spec[1], spec[2], angles, *spec[3:])
    assert m.stats()["sum_eps"] > 1e-6  # truncation is active
    g = m.backward(1.0)
    h = 1e-4
    rng = np.random.default_rng(0)
    idx = rng.choice(angles.size, 24, replace=False)
    fd = np.zeros(idx.size)
    for k, p in enumerate(idx):
        a = angles.copy()
        a[p] += h
        lp = _loss_gpu(T, n, chi, a, spec)
        a[p] -= 2 * h
        lm = _loss_gpu(T, n, chi, a, spec)
        fd[k] = (lp - lm) / (2 * h)
    assert np.linalg.norm(g[idx] - fd) / np.linalg.norm(fd) < 1e-4


def test_autograd_function(T):
    import torch

    n, nl = 5, 2
    angles = W.ansatz_angles(n, nl, 3)
    spec = _spec(n, nl)
    m = T.MPS(n, 32, 0.0)
    a = torch.tensor(angles, dtype=torch.float64, requires_grad=True)
    loss = T.pauli_sum_loss(a, m, spec)
    loss.backward()
    ref = O.parameter_shift(lambda x: W.ansatz_gates(x, n, nl), angles, n, 32, 0.0, spec[4],
                            spec[5])
    assert np.linalg.norm(a.grad.numpy() - ref) / np.linalg.norm(ref) < 1e-8


def test_autograd_two_forwards_on_one_handle(T):
    """A second forward on the same MPS replaces the checkpoints: the second
    loss differentiates correctly and the first one's backward raises."""
    import torch

    n, nl = 5, 2
    spec = _spec(n, nl)
    m = T.MPS(n, 32, 0.0)
    a1 = torch.tensor(W.ansatz_angles(n, nl, 3), dtype=torch.float64, requires_grad=True)
    a2 = torch.tensor(W.ansatz_angles(n, nl, 4), dtype=torch.float64, requires_grad=True)
    l1 = T.pauli_sum_loss(a1, m, spec)
    l2 = T.pauli_sum_loss(a2, m, spec)
    l2.backward()
    ref = O.parameter_shift(lambda x: W.ansatz_gates(x, n, nl), a2.detach().numpy(), n, 32, 0.0,
                            spec[4], spec[5])
    assert np.linalg.norm(a2.grad.numpy() - ref) / np.linalg.norm(ref) < 1e-8
    with pytest.raises(RuntimeError, match="another forward"):
        l1.backward()


# ---------------------------------------------------------------- the 32-qubit, 8-layer ansatz
# (512 angles uniform in [0, 2 pi), Ry/Rz per qubit + CNOT ladder, loss
# sum_i <Z_i Z_{i+1}>)

def _golden_param_shift():
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "ansatz_param_shift.json")
    with open(path) as f:
        return json.load(f)


def test_ansatz32_vs_oracle_parameter_shift(T):
    """At chi_max = 256 the ansatz is not truncated, so the oracle's
    parameter shift is exact; its gradients on 16 seeded angles are stored by
    tests/golden/make_ansatz_param_shift.py (oracle forwards only).  The GPU
    adjoint at the same chi_max must match them within 1e-4 relative (L2 over
    the 16 entries), and the loss within 1e-10."""
    ref = _golden_param_shift()
    n, nl, chi = ref["n"], ref["layers"], ref["chi_max"]
    angles = W.ansatz_angles(n, nl)
    spec = _spec(n, nl)
    m = T.MPS(n, chi, 0.0)
    loss = m.forward_checkpointed(spec[0], spec[1], spec[2], angles, *spec[3:])
    assert m.stats()["sum_eps"] < 1e-12
    assert abs(loss - ref["loss"]) < 1e-10
    g = m.backward(1.0)
    idx = np.array(ref["indices"])
    gr = np.array(ref["grad"])
    assert np.linalg.norm(g[idx] - gr) / np.linalg.norm(gr) < 1e-4


def test_ansatz32_truncated_vs_finite_differences(T):
    """chi_max = 128, where the ansatz truncates in its last layers: the
    adjoint against central differences (h = 1e-4) of the same truncated
    float64 forward on 32 seeded angles, within 1e-4 relative."""
    n, nl, chi = 32, 8, 128
    angles = W.ansatz_angles(n, nl)
    spec = _spec(n, nl)
    m = T.MPS(n, chi, 0.0)
    m.forward_checkpointed(spec[0], spec[1], spec[2], angles, *spec[3:])
    assert m.stats()["sum_eps"] > 1e-8  # truncation is active
    g = m.backward(1.0)
    h = 1e-4
    idx = np.random.default_rng(4141).choice(angles.size, 32, replace=False)
    fd = np.zeros(idx.size)
    for k, p in enumerate(idx):
        a = angles.copy()
        a[p] += h
        lp = _loss_gpu(T, n, chi, a, spec)
        a[p] -= 2 * h
        lm = _loss_gpu(T, n, chi, a, spec)
        fd[k] = (lp - lm) / (2 * h)
    assert np.linalg.norm(g[idx] - fd) / np.linalg.norm(fd) < 1e-4
