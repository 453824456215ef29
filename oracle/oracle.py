"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The GPU library never loads it.

Besides the C core it adds two plain helpers that follow the paper's
definitions on top of the oracle's forward pass:

* ``parameter_shift`` -- gradients of a Pauli-sum loss by the two-term shift
  rule for R_P(t) = exp(-i t P/2) (Mitarai et al., PRA 98, 032309 (2018)).
* ``fidelity`` -- |<a|b>|^2 / (<a|a><b|b>) from two oracle states.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Iterable, List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tnsim_oracle.c")
_LIB = os.path.join(_HERE, "libtnsim_oracle.so")

OK, E_ARG, E_NONLOCAL, E_OVERLAP, E_CAPACITY, E_DEVICE, E_NOCONV = range(7)


def build(force: bool = False) -> str:
    """Compile the oracle (gcc, C99, OpenMP).  Portable x86-64-v3 code."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fcx-fortran-rules", "-fopenmp", "-fPIC",
               "-shared", "-std=gnu99", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None
_lib_path = _LIB


def use_library(path: str | None) -> None:
    """Load a different build of the oracle (used to plant mistakes in a copy
    of the oracle and check that the pins catch them).  None restores it."""
    global _lib, _lib_path
    _lib = None
    _lib_path = path or _LIB


def lib():
    global _lib
    if _lib is None:
        if _lib_path == _LIB and not os.path.exists(_LIB):
            build()
        L = C.CDLL(_lib_path)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.om_create.restype = P
        L.om_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double]
        L.om_destroy.argtypes = [P]
        L.om_n.argtypes = [P]
        L.om_bond_dims.argtypes = [P, ip]
        L.om_stats.argtypes = [P, dp, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int), dp,
                               C.POINTER(C.c_int)]
        L.om_get_site.argtypes = [P, C.c_int, dp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.om_get_lambda.argtypes = [P, C.c_int, dp, C.POINTER(C.c_int)]
        L.om_set_state.argtypes = [P, C.POINTER(dp), C.POINTER(dp), ip]
        L.om_apply_1q.argtypes = [P, C.c_int, dp]
        L.om_apply_2q.argtypes = [P, C.c_int, C.c_int, dp]
        L.om_apply_layer.argtypes = [P, ip, ip, dp, C.c_int]
        L.om_svd.argtypes = [dp, C.c_int, C.c_int, C.c_double, C.c_int, dp, dp, C.POINTER(C.c_int)]
        L.om_truncation.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_double,
                                    C.POINTER(C.c_int), dp, dp]
        L.om_expect_pauli.argtypes = [P, C.c_char_p, dp, dp]
        L.om_norm2.argtypes = [P, dp]
        L.om_overlap.argtypes = [P, P, dp, dp]
        L.om_amplitude.argtypes = [P, C.POINTER(C.c_uint8), dp, dp]
        L.om_statevector.argtypes = [P, dp]
        L.om_sample.argtypes = [P, C.c_int, dp, C.POINTER(C.c_uint8), dp]
        L.om_canonicalize.argtypes = [P, C.c_int]
        L.om_apply_2q_propagate.argtypes = [P, C.c_int, C.c_int, dp]
        L.om_set_threads.argtypes = [C.c_int]
        L.om_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c128(m) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(m, dtype=np.complex128))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what}: status {code}")
        self.code = code


def set_threads(t: int) -> None:
    lib().om_set_threads(int(t))


def threads() -> int:
    return int(lib().om_get_threads())


class OracleMPS:
    """complex128 MPS on the CPU, left-canonical with Schmidt weights per bond."""

    def __init__(self, n: int, chi_max: int, cutoff: float = 0.0, max_sweeps: int = 60,
                 tol: float = 0.0):
        self.n = n
        self._h = lib().om_create(n, chi_max, cutoff, max_sweeps, tol)
        if not self._h:
            raise OracleError(E_ARG, "create")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().om_destroy(h)
            self._h = None

    def _check(self, st: int, what: str) -> None:
        if st != OK:
            raise OracleError(st, what)

    # -- gates
    def apply_1q(self, q: int, u) -> None:
        u = _c128(u).reshape(4)
        self._check(lib().om_apply_1q(self._h, q, _dp(u.view(np.float64))), "apply_1q")

    def apply_2q(self, q0: int, q1: int, g) -> int:
        g = _c128(g).reshape(16)
        st = lib().om_apply_2q(self._h, q0, q1, _dp(g.view(np.float64)))
        return st

    def apply_2q_propagate(self, q0: int, q1: int, g) -> int:
        """Two-qubit gate by bond propagation (distant qubits; neighbours take
        the ordinary two-site path)."""
        gg = _c128(g)
        return lib().om_apply_2q_propagate(self._h, q0, q1, _dp(gg.view(np.float64)))

    def apply(self, gate) -> None:
        q0, q1, m = gate
        if q1 < 0:
            self.apply_1q(q0, m)
        else:
            self._check(self.apply_2q(q0, q1, m), "apply_2q")

    def apply_layer(self, gates: Sequence) -> int:
        ng = len(gates)
        q0 = np.array([g[0] for g in gates], dtype=np.int32)
        q1 = np.array([g[1] for g in gates], dtype=np.int32)
        mats = np.zeros((max(ng, 1), 16), dtype=np.complex128)
        for i, g in enumerate(gates):
            m = _c128(g[2]).reshape(-1)
            mats[i, : m.size] = m
        return lib().om_apply_layer(self._h, q0.ctypes.data_as(C.POINTER(C.c_int32)),
                                    q1.ctypes.data_as(C.POINTER(C.c_int32)),
                                    _dp(mats.view(np.float64)), ng)

    def run(self, gates: Iterable) -> None:
        for g in gates:
            self.apply(g)

    def run_layers(self, layers) -> None:
        for layer in layers:
            self._check(self.apply_layer(layer), "apply_layer")

    # -- state access
    def bond_dims(self) -> np.ndarray:
        out = np.zeros(max(self.n - 1, 1), dtype=np.int32)
        lib().om_bond_dims(self._h, out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out[: self.n - 1]

    def dims(self) -> List[int]:
        return [1] + list(self.bond_dims()) + [1]

    def stats(self) -> dict:
        se, pk, le = C.c_double(), C.c_double(), C.c_double()
        n2 = C.c_int64()
        lk, ls = C.c_int(), C.c_int()
        lib().om_stats(self._h, C.byref(se), C.byref(pk), C.byref(n2), C.byref(lk), C.byref(le),
                       C.byref(ls))
        return {"sum_eps": se.value, "prod_keep": pk.value, "n2q": n2.value, "last_k": lk.value,
                "last_eps": le.value, "last_sweeps": ls.value}

    def site(self, q: int) -> np.ndarray:
        a, b = C.c_int(), C.c_int()
        self._check(lib().om_get_site(self._h, q, None, C.byref(a), C.byref(b)), "site")
        out = np.zeros((a.value, 2, b.value), dtype=np.complex128)
        lib().om_get_site(self._h, q, _dp(out.view(np.float64)), C.byref(a), C.byref(b))
        return out

    def lam(self, bond: int) -> np.ndarray:
        c = C.c_int()
        self._check(lib().om_get_lambda(self._h, bond, None, C.byref(c)), "lambda")
        out = np.zeros(c.value, dtype=np.float64)
        lib().om_get_lambda(self._h, bond, _dp(out), C.byref(c))
        return out

    def set_state(self, sites: Sequence[np.ndarray], lams: Sequence[np.ndarray]) -> None:
        n = self.n
        sites = [np.ascontiguousarray(s, dtype=np.complex128) for s in sites]
        lams = [np.ascontiguousarray(l, dtype=np.float64) for l in lams]
        dims = np.array([1] + [s.shape[2] for s in sites[:-1]] + [1], dtype=np.int32)
        sp = (C.POINTER(C.c_double) * n)(*[_dp(s.view(np.float64)) for s in sites])
        lp = (C.POINTER(C.c_double) * max(n - 1, 1))(*([_dp(l) for l in lams] or [None]))
        self._check(lib().om_set_state(self._h, sp, lp, dims.ctypes.data_as(C.POINTER(C.c_int32))),
                    "set_state")

    # -- readouts
    def expect(self, pauli: str) -> complex:
        re, im = C.c_double(), C.c_double()
        self._check(lib().om_expect_pauli(self._h, pauli.encode(), C.byref(re), C.byref(im)),
                    "expect")
        return complex(re.value, im.value)

    def norm2(self) -> float:
        v = C.c_double()
        lib().om_norm2(self._h, C.byref(v))
        return v.value

    def overlap(self, other: "OracleMPS") -> complex:
        re, im = C.c_double(), C.c_double()
        self._check(lib().om_overlap(self._h, other._h, C.byref(re), C.byref(im)), "overlap")
        return complex(re.value, im.value)

    def amplitude(self, bits: Sequence[int]) -> complex:
        b = np.ascontiguousarray(bits, dtype=np.uint8)
        re, im = C.c_double(), C.c_double()
        self._check(lib().om_amplitude(self._h, b.ctypes.data_as(C.POINTER(C.c_uint8)),
                                       C.byref(re), C.byref(im)), "amplitude")
        return complex(re.value, im.value)

    def sample(self, u: np.ndarray):
        """Perfect sampling: u is shots x n uniforms in [0, 1) (u[shot, q]
        decides qubit q; qubits drawn from n-1 down to 0).  Returns
        (bits uint8 shots x n, log-probability of each drawn string)."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.ndim != 2 or u.shape[1] != self.n:
            raise ValueError("u must be shots x n")
        bits = np.zeros(u.shape, dtype=np.uint8)
        logp = np.zeros(u.shape[0], dtype=np.float64)
        self._check(lib().om_sample(self._h, u.shape[0], _dp(u),
                                    bits.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(logp)),
                    "sample")
        return bits, logp

    def canonicalize(self, truncate: bool = False) -> None:
        """Exact left-canonical form with Schmidt values on every bond, from any
        gauge (two SVD sweeps; the state is normalised).  With truncate, the
        second sweep applies the truncation rule with chi_max and cutoff."""
        self._check(lib().om_canonicalize(self._h, 1 if truncate else 0), "canonicalize")

    def statevector(self) -> np.ndarray:
        out = np.zeros(2 ** self.n, dtype=np.complex128)
        self._check(lib().om_statevector(self._h, _dp(out.view(np.float64))), "statevector")
        return out


def svd(m: np.ndarray, tol: float = 0.0, max_sweeps: int = 60):
    """Oracle Jacobi SVD: returns (U[:, :r], sigma, sweeps), r = min(rows, cols)."""
    m = _c128(m)
    rows, cols = m.shape
    r = min(rows, cols)
    u = np.zeros((r, rows), dtype=np.complex128)  # column-major rows x r
    s = np.zeros(r, dtype=np.float64)
    sw = C.c_int()
    st = lib().om_svd(_dp(m.view(np.float64)), rows, cols, tol, max_sweeps,
                      _dp(u.view(np.float64)), _dp(s), C.byref(sw))
    if st != OK:
        raise OracleError(st, "svd")
    return u.T.copy(), s, sw.value


def truncation(sigma: np.ndarray, rows: int, chi_max: int, cutoff: float):
    """Oracle truncation rule: returns (k, eps, N)."""
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    k, eps, nrm = C.c_int(), C.c_double(), C.c_double()
    st = lib().om_truncation(_dp(s), s.size, rows, chi_max, cutoff, C.byref(k), C.byref(eps),
                             C.byref(nrm))
    if st != OK:
        raise OracleError(st, "truncation")
    return k.value, eps.value, nrm.value


def fidelity(a: OracleMPS, b: OracleMPS) -> float:
    ov = a.overlap(b)
    return abs(ov) ** 2 / (a.norm2() * b.norm2())


def loss_pauli_sum(m: OracleMPS, paulis: Sequence[str], coeffs: Sequence[float]) -> float:
    return float(sum(c * m.expect(p).real for p, c in zip(paulis, coeffs)))


def run_gates(n: int, chi_max: int, cutoff: float, gates: Iterable) -> OracleMPS:
    m = OracleMPS(n, chi_max, cutoff)
    m.run(gates)
    return m


def parameter_shift(make_gates, angles: np.ndarray, n: int, chi_max: int, cutoff: float,
                    paulis: Sequence[str], coeffs: Sequence[float],
                    which: Sequence[int] | None = None) -> np.ndarray:
    """d loss / d angle_p = [f(t_p + pi/2) - f(t_p - pi/2)] / 2 for R_P = exp(-i t P/2).

    ``make_gates(angles)`` returns the gate list.  Exact for an untruncated
    circuit; ``which`` restricts the parameters evaluated."""
    angles = np.asarray(angles, dtype=np.float64)
    idx = range(angles.size) if which is None else which
    g = np.zeros(angles.size)
    for p in idx:
        vals = []
        for sgn in (+1, -1):
            a = angles.copy()
            a[p] += sgn * math.pi / 2
            m = run_gates(n, chi_max, cutoff, make_gates(a))
            vals.append(loss_pauli_sum(m, paulis, coeffs))
        g[p] = 0.5 * (vals[0] - vals[1])
    return g
