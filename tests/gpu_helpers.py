"""Host-side helpers for the GPU tests (test code, not product code)."""
import numpy as np


def dense_from_sites(sites):
    """Dense state from exported site tensors, index x = sum_q b_q 2^q."""
    t = np.ones((1, 1), dtype=np.complex128)
    for a in sites:
        t = np.einsum("xa,asb->sxb", t, a).reshape(-1, a.shape[2])
    return t[:, 0]


def gpu_statevector(m):
    return dense_from_sites([m.site(q) for q in range(m.n)])


def fidelity(a, b):
    return float(abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))


def mps_fidelity_gpu_vs_oracle(g, o, tmp_factory):
    """F between a GPU state and an oracle state: the GPU state is exported to
    a second oracle handle and the overlap is taken by the oracle's transfer
    contraction (complex128)."""
    n = g.n
    sites = [g.site(q) for q in range(n)]
    lams = [g.lam(b) for b in range(n - 1)]
    h = tmp_factory(n)
    h.set_state(sites, lams)
    ov = h.overlap(o)
    return abs(ov) ** 2 / (h.norm2() * o.norm2())
