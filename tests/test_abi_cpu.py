"""C ABI checks that need no GPU: the library loads, exports every symbol
include/tnsim.h declares, and rejects bad input before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2601_04422_amd import tnsim as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tnsim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tnsim_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported():
    lib = T.lib()
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(T._SIGS), "binding signatures out of sync with the header"


def test_arena_bytes_and_config_validation():
    lib = T.lib()
    cfg = T.Config(100, 1024, 1e-12, 3, 1, 0, 0.0, 0)
    big = lib.tnsim_mps_arena_bytes(C.byref(cfg))
    assert big > 3.4e9 / 2  # the sites alone (complex64) take ~1.4 GB
    for bad in (T.Config(1, 8, 0.0, 0, 0, 0, 0.0, 0), T.Config(10, 0, 0.0, 0, 0, 0, 0.0, 0),
                T.Config(10, 8, -1.0, 0, 0, 0, 0.0, 0), T.Config(10, 8, 0.0, 7, 0, 0, 0.0, 0),
                T.Config(10, 8, 0.0, 0, 5, 0, 0.0, 0)):
        assert lib.tnsim_mps_arena_bytes(C.byref(bad)) == 0
    # fewer gates per batch -> smaller arena
    one = T.Config(100, 1024, 1e-12, 0, 0, 0, 0.0, 1)
    assert lib.tnsim_mps_arena_bytes(C.byref(one)) < lib.tnsim_mps_arena_bytes(
        C.byref(T.Config(100, 1024, 1e-12, 0, 0, 0, 0.0, 0)))


def test_create_rejects_bad_arguments_before_device_work():
    lib = T.lib()
    cfg = T.Config(10, 8, 0.0, 0, 0, 0, 0.0, 0)
    h = C.c_void_p()
    need = lib.tnsim_mps_arena_bytes(C.byref(cfg))
    assert lib.tnsim_mps_create(C.byref(cfg), C.c_void_p(256), need - 1, None, C.byref(h)) == \
        T.E_CAPACITY
    assert lib.tnsim_mps_create(C.byref(cfg), None, need, None, C.byref(h)) == T.E_ARG
    assert lib.tnsim_mps_create(C.byref(cfg), C.c_void_p(257), need, None, C.byref(h)) == T.E_ARG
    assert lib.tnsim_mps_create(None, C.c_void_p(256), need, None, C.byref(h)) == T.E_ARG


def _no_gpu():
    import torch

    return torch.cuda.device_count() == 0


@pytest.mark.skipif(not _no_gpu(), reason="only meaningful where no GPU is visible")
def test_create_without_device_reports_device_error():
    lib = T.lib()
    cfg = T.Config(10, 8, 0.0, 0, 0, 0, 0.0, 0)
    h = C.c_void_p()
    need = lib.tnsim_mps_arena_bytes(C.byref(cfg))
    st = lib.tnsim_mps_create(C.byref(cfg), C.c_void_p(1 << 20), need, None, C.byref(h))
    assert st == T.E_DEVICE
    assert not h.value


def test_layerise_greedy():
    g = np.eye(4)
    u = np.eye(2)
    gates = [(0, 1, g), (2, 3, g), (1, 2, g), (0, -1, u), (3, -1, u), (0, 1, g)]
    layers = T.layerise(gates, 4)
    assert [[x[:2] for x in l] for l in layers] == [[(0, 1), (2, 3)], [(1, 2), (0, -1), (3, -1)],
                                                     [(0, 1)]]
    # a layer never reuses a qubit
    for l in layers:
        qs = [q for (a, b, _) in l for q in ((a, b) if b >= 0 else (a,))]
        assert len(qs) == len(set(qs))


def test_status_strings():
    lib = T.lib()
    for code in range(7):
        assert lib.tnsim_status_string(code)


def test_missing_library_fails_loudly(monkeypatch):
    """No CPU fallback: without the built library the binding raises."""
    monkeypatch.setattr(T, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libtnsim.so"))
    monkeypatch.setattr(T, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        T.lib()


def test_sample_workspace_bytes():
    cfg = T.Config(100, 1024, 1e-12, 0, 1, 0, 0.0, 0, 1)
    small = T.lib().tnsim_sample_workspace_bytes(C.byref(cfg), 16)
    big = T.lib().tnsim_sample_workspace_bytes(C.byref(cfg), 4096)
    assert 0 < small < big
    # per-site weights (two chi x chi blocks per site) dominate at few shots
    assert small > 2 * 16 * 1024 * 1024 * 70
    assert T.lib().tnsim_sample_workspace_bytes(C.byref(cfg), 0) == 0
    bad = T.Config(1, 1024, 1e-12, 0, 1, 0, 0.0, 0, 1)
    assert T.lib().tnsim_sample_workspace_bytes(C.byref(bad), 16) == 0


class _StubMPS:
    """Host stand-in for an MPS handle: counts forwards like the binding does,
    so the autograd function's bookkeeping is checked without a device."""

    def __init__(self):
        self.calls = []

    forward_id = property(lambda self: len(self.calls))

    def forward_checkpointed(self, gates, pg, ax, angles, seg, paulis, coeffs):
        self.calls.append(np.array(angles))
        return float(np.sum(np.cos(angles)))

    def backward(self, dloss):
        return -dloss * np.sin(self.calls[-1])


def test_pauli_sum_loss_rejects_a_stale_backward():
    """Two forwards on one handle: the first loss's backward must raise, since
    the handle now holds the second forward's checkpoints."""
    torch = pytest.importorskip("torch")
    m = _StubMPS()
    spec = ([], [], [], [0], [], [])
    a = torch.tensor([0.3, 1.1], dtype=torch.float64, requires_grad=True)
    b = torch.tensor([2.0, -0.5], dtype=torch.float64, requires_grad=True)
    la = T.pauli_sum_loss(a, m, spec)
    lb = T.pauli_sum_loss(b, m, spec)
    lb.backward()
    assert np.allclose(b.grad.numpy(), -np.sin([2.0, -0.5]))
    with pytest.raises(RuntimeError, match="another forward"):
        la.backward()
