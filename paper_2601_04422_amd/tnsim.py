"""Python binding of the tnsim C ABI (include/tnsim.h).

Argument marshalling only: every step of gate application and readout runs
in the HIP library ``libtnsim.so``.  PyTorch provides the device arena and the
stream.  There is no CPU fallback: if the library is missing, or no GPU is
visible, constructing an ``MPS`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtnsim.so")

OK, E_ARG, E_NONLOCAL, E_OVERLAP, E_CAPACITY, E_DEVICE, E_NOCONV = range(7)
PRECISION = {"fp64": 0, "f32acc": 1, "bf16x3": 2, "bf16x6": 3}
STORAGE = {"c128": 0, "c64": 1}


class C128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Config(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("chi_max", C.c_int32), ("cutoff", C.c_double),
                ("precision", C.c_int32), ("storage", C.c_int32),
                ("jacobi_max_sweeps", C.c_int32), ("jacobi_tol", C.c_double),
                ("max_layer_gates", C.c_int32), ("svd_precondition", C.c_int32)]


KERNEL_CLASSES = ["theta", "gram", "eig", "rot", "colnorm", "trunc", "wb_left", "wb_right",
                  "one_qubit", "other", "qr"]
KSTAT_DTYPE = np.dtype([("ms", "<f8"), ("launches", "<i8"), ("flops", "<f8"), ("bytes", "<f8")])
TUNE_BUCKETS = 4  # pair-count classes of the launch-shape table
TUNE_ENTRIES = 2 * TUNE_BUCKETS  # rows per rotation workgroup, then Gram K-split

GATE_DTYPE = np.dtype([("q0", "<i4"), ("q1", "<i4"), ("m", "<c16", (16,))], align=True)
assert GATE_DTYPE.itemsize == 264

# every exported entry point, with its ctypes signature
_P = C.c_void_p
_SIGS = {
    "tnsim_mps_arena_bytes": (C.c_size_t, [C.POINTER(Config)]),
    "tnsim_mps_create": (C.c_int, [C.POINTER(Config), _P, C.c_size_t, _P, C.POINTER(_P)]),
    "tnsim_mps_destroy": (C.c_int, [_P]),
    "tnsim_mps_reset": (C.c_int, [_P]),
    "tnsim_apply_1q": (C.c_int, [_P, C.c_int32, _P]),
    "tnsim_apply_2q": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
    "tnsim_apply_layer": (C.c_int, [_P, _P, C.c_int32]),
    "tnsim_apply_layer_multi": (C.c_int, [_P, _P, _P, C.c_int32]),
    "tnsim_apply_circuit": (C.c_int, [_P, _P, C.c_int32]),
    "tnsim_layerise": (C.c_int, [_P, C.c_int32, C.c_int32, _P, C.POINTER(C.c_int32)]),
    "tnsim_expect_pauli": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]),
    "tnsim_amplitude": (C.c_int, [_P, _P, C.POINTER(C128)]),
    "tnsim_overlap": (C.c_int, [_P, _P, C.POINTER(C128)]),
    "tnsim_mps_copy": (C.c_int, [_P, _P]),
    "tnsim_bond_dims": (C.c_int, [_P, _P]),
    "tnsim_truncation_stats": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_int64)]),
    "tnsim_last_sweeps": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "tnsim_last_batch": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_int32)]),
    "tnsim_sweep_stats": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int32)]),
    "tnsim_export_site": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
    "tnsim_export_lambda": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_int32)]),
    "tnsim_import_state": (C.c_int, [_P, _P, _P, _P]),
    "tnsim_grad_workspace_bytes": (C.c_size_t, [C.POINTER(Config), C.c_int32, C.c_int32,
                                                 C.c_int32]),
    "tnsim_forward_checkpointed": (C.c_int, [_P, _P, C.c_size_t, _P, C.c_int32, _P, _P, _P,
                                             C.c_int32, _P, C.c_int32, _P, _P, C.c_int32,
                                             C.POINTER(C.c_double)]),
    "tnsim_backward": (C.c_int, [_P, C.c_double, _P]),
    "tnsim_sample_workspace_bytes": (C.c_size_t, [C.POINTER(Config), C.c_int32]),
    "tnsim_sample": (C.c_int, [_P, _P, C.c_size_t, C.c_int32, _P, _P, _P]),
    "tnsim_sample_prepare": (C.c_int, [_P, _P, C.c_size_t, C.c_int32]),
    "tnsim_sample_draw": (C.c_int, [_P, _P, C.c_size_t, C.c_int32, _P, _P, _P]),
    "tnsim_profile": (C.c_int, [_P, C.c_int32]),
    "tnsim_profile_read": (C.c_int, [_P, _P]),
    "tnsim_probe_fp64": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "tnsim_autotune": (C.c_int, [_P, _P]),
    "tnsim_set_launch_table": (C.c_int, [_P, _P]),
    "tnsim_canonicalize": (C.c_int, [_P, C.c_int32]),
    "tnsim_apply_2q_propagate": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
    "tnsim_sample_noalloc": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
    "tnsim_qasm_parse": (C.c_int, [C.c_char_p, _P, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), C.c_char_p, C.c_int32]),
    "tnsim_fuse": (C.c_int, [_P, C.c_int32, C.c_int32, _P, C.POINTER(C.c_int32)]),
    "tnsim_status_string": (C.c_char_p, [C.c_int]),
    "tnsim_last_error": (C.c_char_p, [_P]),
}

_lib = None


def lib():
    """Load libtnsim.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"tnsim HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class TnsimError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        msg = lib().tnsim_status_string(code).decode()
        super().__init__(f"{what}: {msg}" + (f" ({detail})" if detail else ""))
        self.code = code


def _c128_array(m, size: int):
    a = np.zeros(size, dtype=np.complex128)
    flat = np.asarray(m, dtype=np.complex128).reshape(-1)
    a[: flat.size] = flat
    return a


def pack_gates(gates: Sequence) -> np.ndarray:
    """[(q0, q1, matrix), ...] -> array of tnsim_gate."""
    arr = np.zeros(len(gates), dtype=GATE_DTYPE)
    for k, (q0, q1, m) in enumerate(gates):
        arr[k]["q0"] = q0
        arr[k]["q1"] = q1
        arr[k]["m"] = _c128_array(m, 16)
    return arr


def unpack_gates(arr: np.ndarray) -> List:
    """array of tnsim_gate -> [(q0, q1, matrix), ...] (2x2 or 4x4 complex)."""
    out = []
    for g in arr:
        m = np.array(g["m"], dtype=np.complex128)
        q0, q1 = int(g["q0"]), int(g["q1"])
        out.append((q0, q1, m[:4].reshape(2, 2).copy() if q1 < 0 else m.reshape(4, 4).copy()))
    return out


def parse_qasm(text: str):
    """OpenQASM 2.0 text -> (n_qubits, [(q0, q1, matrix), ...]) (tnsim_qasm_parse)."""
    b = text.encode()
    n, nq = C.c_int32(), C.c_int32()
    err = C.create_string_buffer(512)
    st = lib().tnsim_qasm_parse(b, None, 0, C.byref(n), C.byref(nq), err, 512)
    if st not in (OK, E_CAPACITY):
        raise TnsimError(st, "qasm_parse", err.value.decode())
    arr = np.zeros(max(n.value, 1), dtype=GATE_DTYPE)
    st = lib().tnsim_qasm_parse(b, arr.ctypes.data, arr.size, C.byref(n), C.byref(nq), err, 512)
    if st != OK:
        raise TnsimError(st, "qasm_parse", err.value.decode())
    return nq.value, unpack_gates(arr[: n.value])


def fuse(gates: Sequence, n_qubits: int) -> List:
    """Gate fusion (tnsim_fuse): the same unitary in fewer gates."""
    arr = pack_gates(gates)
    out = np.zeros(max(len(gates), 1), dtype=GATE_DTYPE)
    n = C.c_int32()
    st = lib().tnsim_fuse(arr.ctypes.data, len(gates), n_qubits, out.ctypes.data, C.byref(n))
    if st != OK:
        raise TnsimError(st, "fuse")
    return unpack_gates(out[: n.value])


def apply_layer_multi(mpss: Sequence["MPS"], layers: Sequence[Sequence]) -> int:
    """Layer k of handle k for every handle, two-qubit gates of all handles in
    shared launches (handle 0 owns the batch; all share one stream)."""
    packed = [pack_gates(l) for l in layers]
    hs = (C.c_void_p * len(mpss))(*[m._h for m in mpss])
    gp = (C.c_void_p * len(mpss))(*[a.ctypes.data for a in packed])
    ng = np.ascontiguousarray([len(l) for l in layers], dtype=np.int32)
    return lib().tnsim_apply_layer_multi(hs, gp, ng.ctypes.data, len(mpss))


def layerise(gates: Sequence, n: int) -> List[List]:
    """Greedy layering of a gate list (library call), returned as layers."""
    arr = pack_gates(gates)
    out = np.zeros(max(len(gates), 1), dtype=np.int32)
    nl = C.c_int32()
    st = lib().tnsim_layerise(arr.ctypes.data, len(gates), n, out.ctypes.data, C.byref(nl))
    if st != OK:
        raise TnsimError(st, "layerise")
    layers: List[List] = [[] for _ in range(nl.value)]
    for g, l in zip(gates, out[: len(gates)]):
        layers[int(l)].append(g)
    return layers


class MPS:
    """An MPS on one GPU, driven through the tnsim C ABI."""

    def __init__(self, n: int, chi_max: int, cutoff: float = 0.0, precision: str = "fp64",
                 storage: str = "c128", jacobi_max_sweeps: int = 0, jacobi_tol: float = 0.0,
                 max_layer_gates: int = 0, device: str = "cuda:0", stream=None,
                 svd_precondition: bool | None = None):
        """svd_precondition: QR-preconditioned Jacobi SVD; None selects it for
        the mixed precisions and leaves the float64 path on plain Jacobi."""
        import torch  # device memory and streams only

        if not torch.cuda.is_available():
            raise RuntimeError("tnsim needs a HIP GPU; none is visible")
        self.n = n
        self.chi_max = chi_max
        self.precision = precision
        self.storage = storage
        if svd_precondition is None:
            svd_precondition = precision != "fp64"
        self.cfg = Config(n, chi_max, cutoff, PRECISION[precision], STORAGE[storage],
                          jacobi_max_sweeps, jacobi_tol, max_layer_gates, int(svd_precondition))
        nbytes = lib().tnsim_mps_arena_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise TnsimError(E_ARG, "arena_bytes")
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            # a non-default stream lets the library capture its Jacobi sweeps in
            # HIP graphs; the default stream runs them as plain launches
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            torch.cuda.synchronize(self.device)
            h = C.c_void_p()
            st = lib().tnsim_mps_create(C.byref(self.cfg), C.c_void_p(self.arena.data_ptr()),
                                        nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != OK:
            raise TnsimError(st, "mps_create", lib().tnsim_last_error(None).decode())
        self._h = h

    @property
    def arena_bytes(self) -> int:
        return self.arena.numel()

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h:
            lib().tnsim_mps_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st: int, what: str) -> None:
        if st != OK:
            raise TnsimError(st, what, lib().tnsim_last_error(self._h).decode())

    # ---------------------------------------------------------------- gates
    def reset(self) -> None:
        self._chk(lib().tnsim_mps_reset(self._h), "reset")

    def apply_1q(self, q: int, u) -> None:
        a = _c128_array(u, 4)
        self._chk(lib().tnsim_apply_1q(self._h, q, a.ctypes.data), "apply_1q")

    def apply_2q(self, q0: int, q1: int, g) -> int:
        a = _c128_array(g, 16)
        return lib().tnsim_apply_2q(self._h, q0, q1, a.ctypes.data)

    def apply_2q_propagate(self, q0: int, q1: int, g) -> int:
        """Two-qubit gate on distant qubits by bond propagation
        (tnsim_apply_2q_propagate); returns the status (E_CAPACITY when the
        window between the qubits cannot hold the propagating bond)."""
        gg = _c128_array(g, 16)
        st = lib().tnsim_apply_2q_propagate(self._h, q0, q1, gg.ctypes.data)
        if st not in (OK, E_CAPACITY):
            self._chk(st, "apply_2q_propagate")
        return st

    def apply(self, gate) -> None:
        q0, q1, m = gate
        if q1 < 0:
            self.apply_1q(q0, m)
        else:
            self._chk(self.apply_2q(q0, q1, m), "apply_2q")

    def apply_layer(self, gates: Sequence) -> int:
        arr = pack_gates(gates)
        return lib().tnsim_apply_layer(self._h, arr.ctypes.data, len(gates))

    def run_layers(self, layers: Iterable[Sequence]) -> None:
        for layer in layers:
            self._chk(self.apply_layer(layer), "apply_layer")

    def apply_circuit(self, gates: Sequence) -> int:
        """A whole circuit in one call: gates start when the gates before them
        on their qubits are done, two-qubit gates of different layers share
        the Jacobi sweeps.  Returns the status."""
        arr = pack_gates(gates)
        return lib().tnsim_apply_circuit(self._h, arr.ctypes.data, len(gates))

    def run_circuit(self, gates: Sequence) -> None:
        self._chk(self.apply_circuit(list(gates)), "apply_circuit")

    def run_gates(self, gates: Iterable) -> None:
        """One gate per call (the per-gate path)."""
        for g in gates:
            self.apply(g)

    # ---------------------------------------------------------------- readouts
    def expect(self, pauli: str) -> complex:
        re, im = C.c_double(), C.c_double()
        self._chk(lib().tnsim_expect_pauli(self._h, pauli.encode(), C.byref(re), C.byref(im)),
                  "expect_pauli")
        return complex(re.value, im.value)

    def amplitude(self, bits: Sequence[int]) -> complex:
        b = np.ascontiguousarray(bits, dtype=np.uint8)
        out = C128()
        self._chk(lib().tnsim_amplitude(self._h, b.ctypes.data, C.byref(out)), "amplitude")
        return complex(out.re, out.im)

    def overlap(self, other: "MPS") -> complex:
        out = C128()
        self._chk(lib().tnsim_overlap(self._h, other._h, C.byref(out)), "overlap")
        return complex(out.re, out.im)

    def norm2(self) -> float:
        return self.overlap(self).real

    def canonicalize(self, truncate: bool = False) -> None:
        """Exact left-canonical form with the Schmidt values on every bond, from
        any gauge; the state is normalised (tnsim_canonicalize)."""
        self._chk(lib().tnsim_canonicalize(self._h, 1 if truncate else 0), "canonicalize")

    def copy_from(self, other: "MPS") -> None:
        self._chk(lib().tnsim_mps_copy(self._h, other._h), "mps_copy")

    # ---------------------------------------------------------------- inspection
    def bond_dims(self) -> np.ndarray:
        out = np.zeros(self.n - 1, dtype=np.int32)
        self._chk(lib().tnsim_bond_dims(self._h, out.ctypes.data), "bond_dims")
        return out

    def stats(self) -> dict:
        se, pk = C.c_double(), C.c_double()
        n2 = C.c_int64()
        self._chk(lib().tnsim_truncation_stats(self._h, C.byref(se), C.byref(pk), C.byref(n2)),
                  "truncation_stats")
        sw = C.c_int32()
        self._chk(lib().tnsim_last_sweeps(self._h, C.byref(sw)), "last_sweeps")
        return {"sum_eps": se.value, "prod_keep": pk.value, "n2q": n2.value,
                "last_sweeps": sw.value}

    def last_batch(self) -> np.ndarray:
        """Rows (i, chiL, chiM, chiR, k, sweeps) for the last apply call."""
        cnt = C.c_int32()
        self._chk(lib().tnsim_last_batch(self._h, None, 0, C.byref(cnt)), "last_batch")
        out = np.zeros((max(cnt.value, 1), 6), dtype=np.int32)
        self._chk(lib().tnsim_last_batch(self._h, out.ctypes.data, cnt.value, C.byref(cnt)),
                  "last_batch")
        return out[: cnt.value]

    # ---------------------------------------------------------------- gradients
    def forward_checkpointed(self, gates: Sequence, param_of_gate: Sequence[int],
                             rot_axis: Sequence[int], angles, segment_start: Sequence[int],
                             paulis: Sequence[str], coeffs: Sequence[float]) -> float:
        """Loss sum_t c_t <P_t> of the circuit from |0...0>, keeping checkpoints
        for ``backward``.  Gates with param_of_gate >= 0 are rotations about
        rot_axis[param] by angles[param] (their matrix is ignored)."""
        import torch

        arr = pack_gates(gates)
        pg = np.ascontiguousarray(param_of_gate, dtype=np.int32)
        ax = np.ascontiguousarray(rot_axis, dtype=np.int32)
        ang = np.ascontiguousarray(angles, dtype=np.float64)
        seg = np.ascontiguousarray(segment_start, dtype=np.int32)
        bounds = list(seg) + [len(gates)]
        max_seg = max(1, max(b - a for a, b in zip(bounds[:-1], bounds[1:])))
        ws = lib().tnsim_grad_workspace_bytes(C.byref(self.cfg), len(seg), max_seg, ang.size)
        if ws == 0:
            raise TnsimError(E_ARG, "grad_workspace_bytes")
        if getattr(self, "_grad_ws", None) is None or self._grad_ws.numel() < ws:
            self._grad_ws = torch.empty(ws, dtype=torch.uint8, device=self.device)
        enc = [p.encode() for p in paulis]
        pp = (C.c_char_p * len(enc))(*enc)
        cf = np.ascontiguousarray(coeffs, dtype=np.float64)
        out = C.c_double()
        self._grad_keep = (arr, pg, ax, ang, seg, enc, pp, cf)
        self._chk(lib().tnsim_forward_checkpointed(
            self._h, C.c_void_p(self._grad_ws.data_ptr()), self._grad_ws.numel(), arr.ctypes.data,
            len(gates), pg.ctypes.data, ax.ctypes.data, ang.ctypes.data, ang.size,
            seg.ctypes.data, seg.size, pp, cf.ctypes.data, cf.size, C.byref(out)),
            "forward_checkpointed")
        self._n_params = ang.size
        # the handle keeps the checkpoints of this forward only: a later
        # forward replaces them, so each forward gets a new id
        self._fwd_id = getattr(self, "_fwd_id", 0) + 1
        return out.value

    @property
    def forward_id(self) -> int:
        """Id of the last forward_checkpointed call (0 before the first)."""
        return getattr(self, "_fwd_id", 0)

    def backward(self, dloss: float = 1.0) -> np.ndarray:
        """Gradient of the loss of the last forward_checkpointed call."""
        g = np.zeros(max(self._n_params, 1), dtype=np.float64)
        self._chk(lib().tnsim_backward(self._h, dloss, g.ctypes.data), "backward")
        return g[: self._n_params]

    # ---------------------------------------------------------------- sampling
    def sample(self, u):
        """Perfect sampling of all qubits (tnsim_sample).  ``u`` holds
        shots x n uniforms in [0, 1) (numpy or a torch tensor; u[i, q] decides
        qubit q of shot i).  Returns (bits, logp) as torch tensors on the
        device: uint8 shots x n, float64 shots."""
        import torch

        ut = torch.as_tensor(u, dtype=torch.float64).to(self.device).contiguous()
        if ut.dim() != 2 or ut.shape[1] != self.n:
            raise ValueError("u must be shots x n")
        shots = ut.shape[0]
        bits = torch.empty((shots, self.n), dtype=torch.uint8, device=self.device)
        logp = torch.empty(shots, dtype=torch.float64, device=self.device)
        if shots == 0:
            return bits, logp
        ws = lib().tnsim_sample_workspace_bytes(C.byref(self.cfg), shots)
        if ws == 0:
            raise TnsimError(E_ARG, "sample_workspace_bytes")
        if getattr(self, "_smp_ws", None) is None or self._smp_ws.numel() < ws:
            self._smp_ws = None
            self._smp_ws = torch.empty(ws, dtype=torch.uint8, device=self.device)
        # the uniforms and outputs were made on torch's stream; the library
        # runs on the handle's stream and returns after it has finished
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._chk(lib().tnsim_sample(self._h, C.c_void_p(self._smp_ws.data_ptr()),
                                     self._smp_ws.numel(), shots, C.c_void_p(ut.data_ptr()),
                                     C.c_void_p(bits.data_ptr()), C.c_void_p(logp.data_ptr())),
                  "sample")
        return bits, logp

    def sample_noalloc(self, u, bits=None, logp=None):
        """The same draws as sample(u) through tnsim_sample_noalloc: the library
        takes its workspace from a fixed device array.  Output tensors may be
        passed in (then nothing is allocated on this call's path)."""
        import torch

        ut = torch.as_tensor(u, dtype=torch.float64).to(self.device).contiguous()
        if ut.dim() != 2 or ut.shape[1] != self.n:
            raise ValueError("u must be shots x n")
        shots = ut.shape[0]
        if bits is None:
            bits = torch.empty((shots, self.n), dtype=torch.uint8, device=self.device)
        if logp is None:
            logp = torch.empty(shots, dtype=torch.float64, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._chk(lib().tnsim_sample_noalloc(self._h, shots, C.c_void_p(ut.data_ptr()),
                                             C.c_void_p(bits.data_ptr()),
                                             C.c_void_p(logp.data_ptr())), "sample_noalloc")
        return bits, logp

    def sample_prepare(self, max_shots: int) -> None:
        """Build the per-site weights once (tnsim_sample_prepare) for later
        sample_draw calls of up to max_shots shots each."""
        import torch

        ws = lib().tnsim_sample_workspace_bytes(C.byref(self.cfg), int(max_shots))
        if ws == 0:
            raise TnsimError(E_ARG, "sample_workspace_bytes")
        self._draw_ws = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self._chk(lib().tnsim_sample_prepare(self._h, C.c_void_p(self._draw_ws.data_ptr()),
                                             self._draw_ws.numel(), int(max_shots)),
                  "sample_prepare")

    def sample_draw(self, u):
        """Draws from the prepared weights; same result as sample(u)."""
        import torch

        ws = getattr(self, "_draw_ws", None)
        if ws is None:
            raise TnsimError(E_ARG, "sample_draw", "call sample_prepare first")
        ut = torch.as_tensor(u, dtype=torch.float64).to(self.device).contiguous()
        if ut.dim() != 2 or ut.shape[1] != self.n:
            raise ValueError("u must be shots x n")
        shots = ut.shape[0]
        bits = torch.empty((shots, self.n), dtype=torch.uint8, device=self.device)
        logp = torch.empty(shots, dtype=torch.float64, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._chk(lib().tnsim_sample_draw(self._h, C.c_void_p(ws.data_ptr()), ws.numel(), shots,
                                          C.c_void_p(ut.data_ptr()), C.c_void_p(bits.data_ptr()),
                                          C.c_void_p(logp.data_ptr())), "sample_draw")
        return bits, logp

    def sample_counts(self, u) -> dict:
        """The drawn strings as a histogram {bit string: count}, the string
        written qubit 0 first (the form in which the paper reports shots)."""
        bits, _ = self.sample(u)
        b = bits.cpu().numpy()
        if b.shape[0] == 0:
            return {}
        rows, counts = np.unique(b, axis=0, return_counts=True)
        return {"".join("01"[int(x)] for x in r): int(c) for r, c in zip(rows, counts)}

    def sweep_stats(self) -> dict:
        g, sm = C.c_int64(), C.c_int64()
        mx = C.c_int32()
        self._chk(lib().tnsim_sweep_stats(self._h, C.byref(g), C.byref(sm), C.byref(mx)),
                  "sweep_stats")
        return {"gates": g.value, "mean": sm.value / max(g.value, 1), "max": mx.value}

    def profile(self, enable: bool) -> None:
        self._chk(lib().tnsim_profile(self._h, 1 if enable else 0), "profile")

    def profile_read(self) -> dict:
        out = np.zeros(len(KERNEL_CLASSES), dtype=KSTAT_DTYPE)
        self._chk(lib().tnsim_profile_read(self._h, out.ctypes.data), "profile_read")
        return {k: {f: out[i][f].item() for f in KSTAT_DTYPE.names}
                for i, k in enumerate(KERNEL_CLASSES)}

    def probe_fp64(self, unit: str, iters: int = 2000) -> float:
        """Attainable float64 TFLOP/s of the device: unit "mfma" (matrix
        cores, v_mfma_f64_16x16x4f64), "valu" (vector FMA), "mixed" (both at
        once, half the wavefronts each) or "mfma4" (v_mfma_f64_4x4x4f64)."""
        out = C.c_double()
        u = {"mfma": 0, "valu": 1, "mixed": 2, "mfma4": 3}[unit]
        self._chk(lib().tnsim_probe_fp64(self._h, u, int(iters), C.byref(out)), "probe_fp64")
        return out.value

    def autotune(self) -> list:
        """Time the rotation and pair-Gram launch shapes on this handle's
        scratch slots and keep the fastest per pair-count class.  Returns the
        table: rows per rotation workgroup for the 4 classes, then the Gram
        K-split for the 4 classes."""
        out = np.zeros(TUNE_ENTRIES, dtype=np.int32)
        self._chk(lib().tnsim_autotune(self._h, out.ctypes.data), "autotune")
        return out.tolist()

    def set_autotune(self, table: Sequence[int]) -> None:
        """Install a launch-shape table (e.g. another handle's autotune result)."""
        t = np.ascontiguousarray(table, dtype=np.int32)
        if t.size != TUNE_ENTRIES:
            raise ValueError(f"launch table needs {TUNE_ENTRIES} entries")
        self._chk(lib().tnsim_set_launch_table(self._h, t.ctypes.data), "set_launch_table")

    def site(self, q: int) -> np.ndarray:
        a, b = C.c_int32(), C.c_int32()
        self._chk(lib().tnsim_export_site(self._h, q, None, C.byref(a), C.byref(b)), "export")
        out = np.zeros((a.value, 2, b.value), dtype=np.complex128)
        self._chk(lib().tnsim_export_site(self._h, q, out.ctypes.data, C.byref(a), C.byref(b)),
                  "export_site")
        return out

    def lam(self, bond: int) -> np.ndarray:
        c = C.c_int32()
        self._chk(lib().tnsim_export_lambda(self._h, bond, None, C.byref(c)), "export")
        out = np.zeros(c.value, dtype=np.float64)
        self._chk(lib().tnsim_export_lambda(self._h, bond, out.ctypes.data, C.byref(c)),
                  "export_lambda")
        return out

    def import_state(self, sites: Sequence[np.ndarray], lams: Sequence[np.ndarray]) -> None:
        n = self.n
        sites = [np.ascontiguousarray(s, dtype=np.complex128) for s in sites]
        lams = [np.ascontiguousarray(l, dtype=np.float64) for l in lams]
        chis = np.array([1] + [s.shape[2] for s in sites[:-1]] + [1], dtype=np.int32)
        sp = (C.c_void_p * n)(*[s.ctypes.data for s in sites])
        lp = (C.c_void_p * max(n - 1, 1))(*([l.ctypes.data for l in lams] or [None]))
        self._chk(lib().tnsim_import_state(self._h, sp, lp, chis.ctypes.data), "import_state")


def _autograd_function():
    import torch

    class PauliSumLoss(torch.autograd.Function):
        """loss(angles) = sum_t c_t <P_t> of a parametrised circuit on an MPS.

        ``forward(angles, mps, spec)`` with spec = (gates, param_of_gate,
        rot_axis, segment_start, paulis, coeffs); the gradient comes from the
        library's hand-written adjoint (tnsim_backward)."""

        @staticmethod
        def forward(ctx, angles, mps, spec):
            gates, pg, ax, seg, paulis, coeffs = spec
            a = angles.detach().to("cpu", torch.float64).numpy()
            loss = mps.forward_checkpointed(gates, pg, ax, a, seg, paulis, coeffs)
            ctx.mps = mps
            ctx.fwd_id = mps.forward_id
            ctx.dev = angles.device
            return torch.tensor(loss, dtype=torch.float64, device=angles.device)

        @staticmethod
        def backward(ctx, grad_out):
            # the handle holds the checkpoints of its last forward only
            if ctx.mps.forward_id != ctx.fwd_id:
                raise RuntimeError(
                    "PauliSumLoss.backward: the MPS ran another forward after this loss was "
                    "computed, so its checkpoints belong to that forward; use one MPS per "
                    "loss that is differentiated")
            g = ctx.mps.backward(float(grad_out))
            return torch.from_numpy(g).to(ctx.dev), None, None

    return PauliSumLoss


def pauli_sum_loss(angles, mps: "MPS", spec):
    """Differentiable Pauli-sum loss (see PauliSumLoss)."""
    return _autograd_function().apply(angles, mps, spec)
