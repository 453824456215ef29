"""Benchmark: two-qubit gates/s at chi = 1024 on one GPU.

Workload: the n=100 circuit of layers "Rx(a), Rz(b) on every qubit, then CNOT
on alternating bonds" at chi_max = 1024, cutoff 1e-12.  Layers 0..P-1 (P = 20
by default) are run untimed with the float64 path to reach saturation (bonds
in the bulk at chi = 1024); that state is the shared starting point of

* the batched mixed path: every gate of a layer in one launch sequence, theta
  contraction and right-site write-back in split-bf16 (or the chosen
  precision), complex64 site storage, float64 Jacobi SVD;
* the per-gate float64 path: one gate per launch sequence, complex128.

A step is one circuit layer (both one-qubit sublayers and the CNOT
sublayer).  ``value`` counts the CNOTs whose three bonds were all 1024 when
applied, over the wall time of the timed steps (inputs already on the GPU).
The per-result error is 1 - F between the two paths' final states.

``cpu_baseline`` times the CPU oracle on one two-qubit gate of the same size
(2048 x 2048 Jacobi SVD) from a seeded random left-canonical input.

One JSON line is printed on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "2q gates/s at χ=1024, batched mixed vs per-gate FP64, fidelity err≤1e-6"
FIDELITY_BOUND = 1e-6
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


# kernel class -> (bound, device kernel name): the Gram and rotation kernels
# are float64 matrix-core contractions, the pair solve and the Householder
# panels float64 vector arithmetic
KERNEL_BOUND = {"rot": ("mfma", "k_rot_mfma3"), "gram": ("mfma", "k_gram_mfma2"),
                "eig": ("alu", "k_eig"), "qr": ("alu", "k_qr_update")}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "jacobi_traffic_chi1024_batched.md")
JACOBI_SRC = os.path.join(ROOT, "paper_2601_04422_amd", "csrc", "k_jacobi.hip")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when that summary was taken on other kernel source."""
    import hashlib
    import re

    try:
        text = open(TRAFFIC_PROFILE).read()
        src = open(JACOBI_SRC, "rb").read()
    except OSError:
        return None
    m = re.search(r"sha256 `([0-9a-f]{64})`", text)
    if not m or m.group(1) != hashlib.sha256(src).hexdigest():
        return None
    m = re.search(rf"traffic_bytes_per_launch {kernel} (\d+)", text)
    return int(m.group(1)) if m else None


def roofline(prof):
    """Roofline entry of the kernel class with the most time: algorithmic
    flops (device work counters) over its HIP-event time, against the float64
    peak (matrix cores for the contractions, vector units otherwise)."""
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    launches = max(d["launches"], 1)
    bound, kname = KERNEL_BOUND.get(dom, ("alu", dom))
    if d["flops"] > 0:
        achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
        out = {"bound": bound, "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": achieved / FP64_PEAK_TFLOPS, "traffic": measured_traffic(kname),
               "kernel": kname, "launches": d["launches"], "avg_launch_ms": d["ms"] / launches,
               "flops_per_launch": d["flops"] / launches,
               "algorithmic_bytes_per_launch": d["bytes"] / launches}
        if bound == "mfma":
            # the matrix-core kernels form a complex product from three real
            # ones (Gauss), so the units execute 3/4 of the algorithmic flops
            out["executed_frac"] = 0.75 * achieved / FP64_PEAK_TFLOPS
        return out
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname), "kernel": kname,
            "launches": d["launches"], "avg_launch_ms": d["ms"] / launches}


BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3


def kernel_rates(prof, precision):
    """Achieved algorithmic rates per kernel class over the timed region:
    TFLOP/s against the peak of the unit the class runs on, and GB/s against
    HBM.  The merge and the right-site write-back count their complex
    products once (the split products on bf16 matrix cores are not counted)."""
    unit = {"theta": precision, "wb_right": precision}
    out = {}
    for k, v in prof.items():
        if not v["launches"] or v["ms"] <= 0:
            continue
        sec = v["ms"] * 1e-3
        r = {"ms": round(v["ms"], 3)}
        if v["flops"] > 0:
            tf = v["flops"] / sec / 1e12
            pk = FP64_PEAK_TFLOPS
            if unit.get(k) in ("bf16x3", "bf16x6"):
                pk = BF16_PEAK_TFLOPS
            elif unit.get(k) == "f32acc":
                pk = FP32_PEAK_TFLOPS
            r.update({"tflops": round(tf, 2), "peak_tflops": pk, "frac": round(tf / pk, 3)})
        if v["bytes"] > 0:
            gb = v["bytes"] / sec / 1e9
            r.update({"gbs": round(gb, 1), "hbm_frac": round(gb / HBM_PEAK_GBS, 3)})
        out[k] = r
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prep-layers", type=int, default=20)
    ap.add_argument("--precision", default=None, choices=["fp64", "f32acc", "bf16x3", "bf16x6"],
                    help="merge and write-back arithmetic of the batched path (default: fp64 "
                         "for the headline, bf16x6 for the batch, nonlocal, sample and qasm "
                         "workloads)")
    ap.add_argument("--storage", default=None, choices=["c128", "c64"],
                    help="site storage (default: c128 for the headline, c64 for the others)")
    ap.add_argument("--profile-steps", type=int, default=-1,
                    help="layers of the profiled pass (default: all timed layers)")
    ap.add_argument("--chi", type=int, default=1024)
    ap.add_argument("--jacobi-tol", type=float, default=0.0,
                    help="relative Jacobi tolerance of the batched path (0: the library default)")
    ap.add_argument("--no-pergate", action="store_true")
    ap.add_argument("--variants", default="fp64_c128,fp64_c128_tol30,fp64_c128_tol27,bf16x6_c64,"
                                          "bf16x6_c64_local,fp64_c128_tol30_local",
                    help="fidelity workload: batched variants to follow (see bench_fidelity)")
    ap.add_argument("--circuit", action="store_true",
                    help="batched path: the timed layers as one dependency-scheduled "
                         "circuit call instead of one call per sublayer")
    ap.add_argument("--shots", type=int, default=4096, help="sample workload: shots per call")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="oracle threads of the secondary workloads")
    ap.add_argument("--workload", default="chi1024",
                    choices=["chi1024", "wide", "ansatz", "batch", "nonlocal", "sample", "qasm",
                             "fidelity", "calib", "propagate", "canonical", "peak"],
                    help="chi1024: the headline metric; the others measure the secondary "
                         "workloads (one JSON line each)")
    return ap.parse_args()


def circuit_layers(n_layers):
    from paper_2601_04422_amd import workloads as W

    sub = W.config_chi1024(n_layers).layers  # 3 sublayers per circuit layer
    return [sub[3 * l: 3 * l + 3] for l in range(n_layers)]


def count_full(m, cnot_layer, chi):
    d = [1] + list(m.bond_dims()) + [1]
    return sum(1 for (q0, q1, _) in cnot_layer if d[q0] == chi and d[q0 + 1] == chi and d[q0 + 2] == chi)


def run_layer_batched(m, layer):
    for sub in layer:
        st = m.apply_layer(sub)
        if st != 0:
            raise RuntimeError(f"apply_layer failed with status {st}")


def run_layer_pergate(m, layer):
    for sub in layer:
        m.run_gates(sub)


def cpu_baseline(threads, chi):
    """Oracle time for one chi x chi x chi two-qubit gate (seeded random input)."""
    from oracle import oracle as O
    from paper_2601_04422_amd import workloads as W

    O.set_threads(threads)
    rng = np.random.default_rng(77)
    dims = [1, chi, chi, chi, 1]
    sites = [rng.standard_normal((1, 2, chi)) + 0j,
             W.random_isometry(rng, 2 * chi, chi).reshape(chi, 2, chi),
             W.random_isometry(rng, 2 * chi, chi).reshape(chi, 2, chi),
             rng.standard_normal((chi, 2, 1)) + 0j]
    lams = [W.schmidt_profile(rng, chi) for _ in range(3)]
    m = O.OracleMPS(4, chi, 1e-12)
    m.set_state(sites, lams)
    g = W.cnot() @ np.kron(W.rz(0.7) @ W.rx(1.3), W.rz(2.1) @ W.rx(0.4))
    t0 = time.perf_counter()
    st = m.apply_2q(1, 2, g)
    dt = time.perf_counter() - t0
    if st != 0:
        raise RuntimeError(f"oracle gate failed: {st}")
    s = m.stats()
    return {"value": 1.0 / dt, "unit": "2q gates/s", "cores": O.threads(), "kind": "oracle",
            "sample": f"1 two-qubit gate at chiL=chiM=chiR={chi} (M is {2*chi}x{2*chi}, "
                      f"Jacobi {s['last_sweeps']} sweeps, kept {s['last_k']}) on a seeded random "
                      f"left-canonical input; {dt:.1f} s"}


def bench_wide(args):
    """n=64 Haar brickwork, depth 20, chi_max=256, cutoff 1e-10, complex64 with the
    float32 matrix-core contraction, one batched launch sequence per layer;
    per-site <Z> against the float64 path."""
    import torch

    from paper_2601_04422_amd import tnsim as T
    from paper_2601_04422_amd import workloads as W

    cfg = W.config_wide()
    m = T.MPS(cfg.n, cfg.chi_max, cfg.cutoff, precision="f32acc", storage="c64")
    ref = T.MPS(cfg.n, cfg.chi_max, cfg.cutoff, precision="fp64", storage="c128")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.run_layers(cfg.layers)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    ref.run_layers(cfg.layers)
    torch.cuda.synchronize()
    dt_ref = time.perf_counter() - t1
    zs = []
    for q in range(cfg.n):
        s = ["I"] * cfg.n
        s[q] = "Z"
        zs.append((m.expect("".join(s)).real, ref.expect("".join(s)).real))
    zerr = max(abs(a - b) for a, b in zs)
    fid = abs(m.overlap(ref)) ** 2 / (m.norm2() * ref.norm2())
    return {"metric": "2q gates/s, n=64 brickwork chi_max=256", "value": cfg.n2q() / dt,
            "unit": "2q gates/s", "n_gpus": 1, "steps": len(cfg.layers), "warmup": 0,
            "ms_per_step": 1e3 * dt / len(cfg.layers), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32acc contraction, f64 svd",
            "data": "synthetic",
            "config": {"workload": cfg.name + ", cutoff 1e-10, complex64"},
            "fp64_path_gates_per_s": cfg.n2q() / dt_ref,
            "max_abs_dZ_vs_fp64": zerr, "fidelity_err_vs_fp64": 1 - fid,
            "sum_eps": m.stats()["sum_eps"]}


def bench_ansatz(args):
    """Gradient of sum_i <Z_i Z_i+1> for the n=32, 8-layer Ry/Rz + CNOT-ladder
    ansatz at chi_max=128: forward (checkpointed) + adjoint backward time and
    the gradient error against central finite differences on a sample."""
    import torch

    from paper_2601_04422_amd import tnsim as T
    from paper_2601_04422_amd import workloads as W

    n, nl, chi = 32, 8, 128
    angles = W.ansatz_angles(n, nl)
    qs, ps, axes = W.ansatz_structure(n, nl)
    gates = [(q0, q1, W.cnot() if q1 >= 0 else np.eye(2)) for (q0, q1) in qs]
    rot_axis = np.zeros(angles.size, dtype=np.int32)
    for p, ax in zip(ps, axes):
        if p >= 0:
            rot_axis[p] = ax
    per_layer = 2 * n + n - 1
    seg = [l * per_layer for l in range(nl)]
    paulis = W.zz_chain(n)
    coeffs = [1.0] * len(paulis)
    m = T.MPS(n, chi, 0.0)
    m.forward_checkpointed(gates, ps, rot_axis, angles, seg, paulis, coeffs)  # warm-up
    m.backward(1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = m.forward_checkpointed(gates, ps, rot_axis, angles, seg, paulis, coeffs)
    t1 = time.perf_counter()
    g = m.backward(1.0)
    t2 = time.perf_counter()
    sum_eps = m.stats()["sum_eps"]
    rng = np.random.default_rng(0)
    idx = rng.choice(angles.size, 8, replace=False)
    h = 1e-4
    fd = []
    for p in idx:
        a = angles.copy()
        a[p] += h
        lp = T.MPS(n, chi, 0.0).forward_checkpointed(gates, ps, rot_axis, a, seg, paulis, coeffs)
        a[p] -= 2 * h
        lm = T.MPS(n, chi, 0.0).forward_checkpointed(gates, ps, rot_axis, a, seg, paulis, coeffs)
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    err = float(np.linalg.norm(g[idx] - fd) / np.linalg.norm(fd))
    return {"metric": "forward+backward time, n=32 8-layer ansatz, 512 angles, chi_max=128",
            "value": t2 - t0, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": 1e3 * (t2 - t0), "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "Ry,Rz per qubit + CNOT ladder, 8 layers, loss sum Z_i Z_i+1"},
            "forward_s": t1 - t0, "backward_s": t2 - t1, "loss": loss, "sum_eps": sum_eps,
            "grad_rel_err_vs_fd_sample": err}


def bench_batch(args):
    """256 independent brickwork circuits of uneven n, depth and chi_max,
    complex64 + split-bf16 contraction, all gates of a layer step of all
    circuits in shared launches; aggregate gates/s and per-circuit fidelity
    against the oracle for the small circuits."""
    import torch

    from oracle import oracle as O
    from paper_2601_04422_amd import tnsim as T
    from paper_2601_04422_amd import workloads as W

    circs = sorted(W.config_batch(), key=lambda c: -c.depth)
    ms = []
    for k, c in enumerate(circs):
        mlg = 8192 if k == 0 else (4 if c.chi_max >= 256 else 8)
        ms.append(T.MPS(c.n, c.chi_max, 1e-10, precision=args.precision, storage="c64",
                        max_layer_gates=mlg))
    total = sum(sum(len(l) for l in c.layers) for c in circs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(max(c.depth for c in circs)):
        act = [k for k, c in enumerate(circs) if t < c.depth]
        st = T.apply_layer_multi([ms[k] for k in act], [circs[k].layers[t] for k in act])
        if st != 0:
            raise RuntimeError(f"apply_layer_multi failed: {st}")
        log(f"batch step {t}: {len(act)} circuits ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # oracle fidelity for the circuits it finishes quickly
    O.set_threads(args.cpu_threads)
    fids = []
    t_or = time.perf_counter()
    for k in sorted(range(len(circs)), key=lambda k: circs[k].chi_max * circs[k].n):
        c = circs[k]
        if c.chi_max > 64 or time.perf_counter() - t_or > 60:
            break
        o = O.OracleMPS(c.n, c.chi_max, 1e-10)
        o.run_layers(c.layers)
        sites = [ms[k].site(q) for q in range(c.n)]
        lams = [ms[k].lam(b) for b in range(c.n - 1)]
        h = O.OracleMPS(c.n, 4096)
        h.set_state(sites, lams)
        fids.append(1 - abs(h.overlap(o)) ** 2 / (h.norm2() * o.norm2()))
    return {"metric": "aggregate 2q gates/s, 256 ragged brickwork circuits", "value": total / dt,
            "unit": "2q gates/s", "n_gpus": 1, "steps": max(c.depth for c in circs),
            "warmup": 0, "ms_per_step": 1e3 * dt / max(c.depth for c in circs),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": f"{args.precision} contraction, f64 svd", "data": "synthetic",
            "config": {"workload": "256 circuits: n U{16..96}, depth U{8..24}, chi_max in "
                                   "{32,64,128,256,512}, cutoff 1e-10, complex64"},
            "total_2q_gates": total,
            "oracle_checked_circuits": len(fids),
            "max_fidelity_err_vs_oracle": max(fids) if fids else None}


def oracle_rate(gates, n, chi, cutoff, threads, budget_s=20.0):
    """The CPU oracle on the first gates of a circuit until budget_s has
    passed: two-qubit gates per second (the early gates meet smaller bonds,
    so this flatters the CPU)."""
    from oracle import oracle as O

    O.set_threads(threads)
    o = O.OracleMPS(n, chi, cutoff)
    t0 = time.perf_counter()
    k = done = 0
    for g in gates:
        o.apply(g)
        k += 1
        done += g[1] >= 0
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "2q gates/s", "cores": O.threads(), "kind": "oracle",
            "sample": f"first {k} of {len(gates)} gates ({done} two-qubit), {dt:.1f} s"}


def bench_nonlocal(args):
    """Gates on distant qubits (SWAP chains): n=48, 400 gates, 60% two-qubit
    gates (Haar U(4)) on random pairs up to 8 apart, chi_max=128, cutoff 1e-10.
    The mixed path takes the whole circuit in one scheduled call; the float64
    path one gate per call.  Rates count the circuit's two-qubit gates (not
    the SWAPs they expand into)."""
    import torch

    from paper_2601_04422_amd import tnsim as T
    from paper_2601_04422_amd import workloads as W

    n, chi, count = 48, 128, 400
    rng = np.random.default_rng(1006)
    gates = []
    for _ in range(count):
        if rng.random() < 0.4:
            q = int(rng.integers(0, n))
            gates.append((q, -1, W.rot("XYZ"[int(rng.integers(0, 3))], rng.uniform(0, 2 * np.pi))))
        else:
            a = int(rng.integers(0, n))
            d = int(rng.integers(1, 9)) * (1 if rng.random() < 0.5 else -1)
            b = min(max(a + d, 0), n - 1)
            if b == a:
                b = a + 1 if a + 1 < n else a - 1
            gates.append((a, b, W.haar_u4(rng)))
    n2q = sum(1 for g in gates if g[1] >= 0)
    swaps = sum(2 * (abs(g[0] - g[1]) - 1) for g in gates if g[1] >= 0)
    m = T.MPS(n, chi, 1e-10, precision=args.precision, storage=args.storage)
    ref = T.MPS(n, chi, 1e-10, precision="fp64", storage="c128")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.run_circuit(gates)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    ref.run_gates(gates)
    torch.cuda.synchronize()
    dt_ref = time.perf_counter() - t1
    fid = abs(m.overlap(ref)) ** 2 / (m.norm2() * ref.norm2())
    cpu = None if args.no_cpu else oracle_rate(gates, n, chi, 1e-10, args.cpu_threads)
    return {"metric": "non-local 2q gates/s, n=48 random pairs up to 8 apart, chi_max=128",
            "value": n2q / dt, "unit": "2q gates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": f"{args.precision} contraction, f64 svd",
            "data": "synthetic",
            "config": {"workload": f"{count} gates, {n2q} two-qubit ({swaps} SWAPs added), "
                                   f"cutoff 1e-10, {args.storage}"},
            "fp64_per_gate_gates_per_s": n2q / dt_ref, "fidelity_err_vs_fp64": 1 - fid,
            "max_bond": int(max(m.bond_dims())), "cpu_baseline": cpu}


def bench_propagate(args):
    """Distant two-qubit gates by bond propagation against SWAP chains: n=48,
    chi_max=256, cutoff 1e-10, float64; 300 gates, 40% one-qubit rotations
    and 60% CNOTs (operator rank 2) on random pairs 2..8 apart, one call per
    gate on both handles.  A propagation whose window cannot hold the
    propagating bond (E_CAPACITY) takes the SWAP chain instead; the line
    counts both.  Rates count the circuit's two-qubit gates."""
    import torch

    from paper_2601_04422_amd import tnsim as T
    from paper_2601_04422_amd import workloads as W

    n, chi, count = 48, 256, 300
    rng = np.random.default_rng(1008)
    gates = []
    for _ in range(count):
        if rng.random() < 0.4:
            q = int(rng.integers(0, n))
            gates.append((q, -1, W.rot("XYZ"[int(rng.integers(0, 3))], rng.uniform(0, 2 * np.pi))))
        else:
            a = int(rng.integers(0, n))
            d = int(rng.integers(2, 9)) * (1 if rng.random() < 0.5 else -1)
            b = min(max(a + d, 0), n - 1)
            if abs(b - a) < 2:
                b = a + 2 if a + 2 < n else a - 2
            gates.append((a, b, W.cnot()))
    n2q = sum(1 for g in gates if g[1] >= 0)
    sw = T.MPS(n, chi, 1e-10)
    pr = T.MPS(n, chi, 1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sw.run_gates(gates)
    torch.cuda.synchronize()
    t_sw = time.perf_counter() - t0
    fallback = 0
    t0 = time.perf_counter()
    for g in gates:
        if g[1] < 0:
            pr.apply(g)
        elif pr.apply_2q_propagate(g[0], g[1], g[2]) != T.OK:
            fallback += 1
            pr.apply(g)
    torch.cuda.synchronize()
    t_pr = time.perf_counter() - t0
    fid = abs(sw.overlap(pr)) ** 2 / (sw.norm2() * pr.norm2())
    return {"metric": "distant 2q gates/s by bond propagation, n=48 CNOTs 2..8 apart, chi_max=256",
            "value": n2q / t_pr, "unit": "2q gates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": 1e3 * t_pr, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{count} gates, {n2q} CNOTs on pairs 2..8 apart, cutoff 1e-10"},
            "swap_chain_gates_per_s": n2q / t_sw, "propagation_fell_back_to_swaps": fallback,
            "one_minus_F_propagation_vs_swaps": 1 - fid,
            "sum_eps": {"propagation": pr.stats()["sum_eps"], "swaps": sw.stats()["sum_eps"]},
            "max_bond": int(max(pr.bond_dims()))}


def bench_canonical(args):
    """Canonical form of the chi=1024 benchmark state: the n=100 benchmark
    circuit runs --prep-layers layers (float64, batched), then each timed step
    is one tnsim_canonicalize call (two sweeps of 99 two-site decompositions,
    one after the other).  Reports the gauge defect the call removes (largest
    deviation of a site from left-canonical before and after)."""
    import torch

    from paper_2601_04422_amd import tnsim as T

    n, chi = 100, args.chi
    layers = circuit_layers(args.prep_layers)
    m = T.MPS(n, chi, 1e-12, precision="fp64", storage="c128", svd_precondition=True,
              stream=torch.cuda.Stream())
    for l in range(args.prep_layers):
        run_layer_batched(m, layers[l])
    torch.cuda.synchronize()

    def defect():
        worst = 0.0
        for q in range(n - 1):
            a = m.site(q)
            a = a.reshape(-1, a.shape[2])
            worst = max(worst, float(np.max(np.abs(a.conj().T @ a - np.eye(a.shape[1])))))
        return worst

    before = defect()
    times = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.canonicalize()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return {"metric": f"canonicalisation time, n=100 chi={chi} benchmark state",
            "value": min(times), "unit": "s", "n_gpus": 1, "steps": len(times), "warmup": 0,
            "ms_per_step": 1e3 * min(times), "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"state after {args.prep_layers} layers of the benchmark "
                                   f"circuit, chi_max={chi}"},
            "seconds_each": times, "left_canonical_defect": {"before": before, "after": defect()},
            "bonds_at_chi": int(sum(1 for d in m.bond_dims() if d == chi))}


def bench_sample(args):
    """Perfect sampling from the chi=1024 benchmark state: the n=100 benchmark
    circuit runs on the mixed path (untimed, --prep-layers layers) until the
    bonds saturate, then each timed step draws --shots strings in one call,
    uniforms already on the GPU.  The first strings' log-probabilities are
    checked against |<x|psi>|^2 / <psi|psi> from the amplitude path."""
    import torch

    from paper_2601_04422_amd import tnsim as T

    n, chi, S = 100, args.chi, args.shots
    layers = circuit_layers(args.prep_layers)
    m = T.MPS(n, chi, 1e-12, precision=args.precision, storage=args.storage)
    t0 = time.perf_counter()
    for l in range(args.prep_layers):
        run_layer_batched(m, layers[l])
        log(f"prep layer {l}: max chi {int(max(m.bond_dims()))}")
    torch.cuda.synchronize()
    log(f"state ready: max chi {int(max(m.bond_dims()))}, "
        f"{sum(1 for d in m.bond_dims() if d == chi)} bonds at {chi} "
        f"({time.perf_counter() - t0:.1f} s)")
    rng = np.random.default_rng(2024)
    u = torch.as_tensor(rng.random((S, n)), device=m.device)
    for _ in range(args.warmup):
        m.sample(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bits, logp = m.sample(u)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the same draws from weights built once (tnsim_sample_prepare / _draw)
    m.sample_prepare(S)
    m.sample_draw(u)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        m.sample_draw(u)
    torch.cuda.synchronize()
    dt_draw = (time.perf_counter() - t1) / args.steps
    b = bits.cpu().numpy()
    lp = logp.cpu().numpy()
    nrm = m.norm2()
    err = max(abs(lp[i] - math.log(abs(m.amplitude(b[i])) ** 2 / nrm)) for i in range(8))
    # algorithmic float64 work of one call (8 flops per complex multiply-add):
    # per-site weights M_q^s = A_q^{sH} E_q A_q^s (4 chi^3), node weights
    # [M^0; M^1] V (2 chi_R^2 m_q) and next nodes A^s v (chi_L chi_R m'_q), with
    # m_q the distinct suffixes before drawing qubit q and m'_q after
    d = [1] + [int(x) for x in m.bond_dims()] + [1]
    env = sum(8.0 * (d[q] ** 2 * 2 * d[q + 1] + 2 * d[q] * d[q + 1] ** 2) for q in range(n))
    distinct = [len({r.tobytes() for r in b[:, q:]}) for q in range(n)] + [1]
    nw = ny = 0.0
    for q in range(n - 1, -1, -1):
        ny += 8.0 * 2 * d[q + 1] ** 2 * distinct[q + 1]
        nw += 8.0 * d[q] * d[q + 1] * distinct[q]
    return {"metric": "shots/s, perfect sampling of all 100 qubits at chi=1024",
            "value": S / dt, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * dt, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"benchmark circuit state after {args.prep_layers} layers "
                                   f"({args.precision}, {args.storage}), {S} shots per call"},
            "distinct_strings": int(len({tuple(r) for r in b})),
            "draw_only_shots_per_s": S / dt_draw,
            "flops_per_call": {"environments": env, "node_products": nw, "node_weights": ny},
            "tflops_per_s": (env + nw + ny) / dt / 1e12,
            "max_abs_logp_err_vs_amplitude": err}


def bench_qasm(args):
    """A circuit read from OpenQASM: 20 Trotter steps of a Heisenberg chain
    on 64 qubits (rxx, ryy, rzz on every bond, then rz fields), chi_max=256,
    cutoff 1e-10, through the dependency scheduler, as parsed and after gate
    fusion (three two-qubit gates per bond and step become one)."""
    import torch

    from paper_2601_04422_amd import tnsim as T
    from paper_2601_04422_amd import workloads as W

    n, chi = 64, 256
    text = W.heisenberg_qasm(n, 20)
    t0 = time.perf_counter()
    nq, gates = T.parse_qasm(text)
    t_parse = time.perf_counter() - t0
    t0 = time.perf_counter()
    fused = T.fuse(gates, nq)
    t_fuse = time.perf_counter() - t0
    res = {}
    for name, circ in (("parsed", gates), ("fused", fused)):
        m = T.MPS(n, chi, 1e-10, precision=args.precision, storage=args.storage)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.run_circuit(circ)
        torch.cuda.synchronize()
        res[name] = (m, time.perf_counter() - t0, sum(1 for g in circ if g[1] >= 0))
        log(f"{name}: {res[name][2]} two-qubit gates, {res[name][1]:.2f} s, "
            f"max chi {int(max(m.bond_dims()))}")
    a, b = res["parsed"][0], res["fused"][0]
    fid = abs(a.overlap(b)) ** 2 / (a.norm2() * b.norm2())
    n2q = res["parsed"][2]
    cpu = None
    if not args.no_cpu:  # the oracle on the fused circuit, rate in gates of the parsed one
        cpu = oracle_rate(fused, n, chi, 1e-10, args.cpu_threads)
        cpu["value"] *= n2q / max(1, res["fused"][2])
        cpu["unit"] = "2q gates/s (of the parsed circuit)"
    return {"metric": "circuit 2q gates/s, 64-qubit Heisenberg Trotter circuit from OpenQASM, fused",
            "value": n2q / res["fused"][1], "unit": "2q gates/s (of the parsed circuit)",
            "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * res["fused"][1],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": f"{args.precision} contraction, f64 svd", "data": "synthetic",
            "config": {"workload": f"heisenberg n={n}, 20 steps, dt=0.1, chi_max={chi}, "
                                   f"cutoff 1e-10, {args.storage}"},
            "parse_ms": 1e3 * t_parse, "fuse_ms": 1e3 * t_fuse,
            "two_qubit_gates": {"parsed": n2q, "fused": res["fused"][2]},
            "seconds": {"parsed": res["parsed"][1], "fused": res["fused"][1]},
            "fused_vs_parsed_1_minus_F": 1 - fid,
            "max_bond": int(max(b.bond_dims())), "cpu_baseline": cpu}


def host_cpu():
    """Threads the oracle may use on this host and the CPU model."""
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS") or visible)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return min(threads, visible), visible, model


def snapshot_gate(m, layer, chi):
    """Inputs of the first two-qubit gate of `layer` whose three bonds are all
    at chi, exported from handle `m` (the state before the layer): the one-qubit
    sublayers of the layer are folded into the gate, G (U_i x U_i+1)."""
    from paper_2601_04422_amd import workloads as W

    d = [1] + list(m.bond_dims()) + [1]
    u = {}
    for sub in layer[:-1]:
        for (q, q1, g) in sub:
            if q1 < 0:
                u[q] = np.asarray(g) @ u.get(q, np.eye(2))
    for (i, j, g) in layer[-1]:
        if d[i] == chi and d[i + 1] == chi and d[i + 2] == chi:
            gg = np.asarray(g) @ np.kron(u.get(i, np.eye(2)), u.get(j, np.eye(2)))
            lams = [m.lam(i - 1) if i >= 1 else np.ones(1), m.lam(i), m.lam(i + 1)]
            return i, m.site(i), m.site(i + 1), lams, gg
    raise RuntimeError("no gate at full bond dimension in the layer")


def cpu_baseline_snapshot(gate_inputs, chi, threads, cpus_visible, model):
    """The CPU oracle on one two-qubit gate of the benchmark circuit: sites i,
    i+1 and the Schmidt weights around them exported from the GPU state at the
    start of the timed layers, in a 4-site chain whose outer sites only fix the
    shapes (the gate reads sites i, i+1 and lambda_{i+1})."""
    from oracle import oracle as O

    i, a0, a1, lams, g = gate_inputs
    O.set_threads(threads)
    rng = np.random.default_rng(77)
    chiL, chiR = a0.shape[0], a1.shape[2]
    sites = [rng.standard_normal((1, 2, chiL)) + 0j, a0, a1, rng.standard_normal((chiR, 2, 1)) + 0j]
    o = O.OracleMPS(4, chi, 1e-12)
    o.set_state(sites, lams)
    t0 = time.perf_counter()
    st = o.apply_2q(1, 2, g)
    dt = time.perf_counter() - t0
    if st != 0:
        raise RuntimeError(f"oracle gate failed: {st}")
    s = o.stats()
    return {"value": 1.0 / dt, "unit": "2q gates/s", "cores": O.threads(), "kind": "oracle",
            "cpu_model": model, "host_cpus_visible": cpus_visible,
            "sample": f"1 two-qubit gate of the benchmark circuit (CNOT on ({i},{i + 1}) with the "
                      f"layer's Rx,Rz folded in) from the GPU state at the start of the timed "
                      f"layers: chiL=chiM=chiR={chi}, M is {2 * chiL}x{2 * chiR}, Jacobi "
                      f"{s['last_sweeps']} sweeps, kept {s['last_k']}; {dt:.1f} s"}


def bench_fidelity(args):
    """Per-layer 1 - F of batched variants against the per-gate float64 path,
    every variant starting from the shared float64 snapshot at layer
    --prep-layers and running the next --steps layers (--variants picks
    them): split-bf16 merge and write-back with complex64 or complex128
    sites, the float64 Jacobi tolerance on complex64 sites, float64
    throughout with the default tolerance or with 2^-30 or 2^-27; a name
    ending in _local restarts every layer from the per-gate state, i.e. it
    measures the error one layer adds."""
    import torch

    from paper_2601_04422_amd import tnsim as T

    n, chi, P, K = 100, args.chi, args.prep_layers, args.steps
    layers = circuit_layers(P + K)
    ref = T.MPS(n, chi, 1e-12, precision="fp64", storage="c128")
    for l in range(P):
        run_layer_batched(ref, layers[l])
    torch.cuda.synchronize()
    every = {"bf16x6_c64": dict(precision="bf16x6", storage="c64"),
             "bf16x6_c128": dict(precision="bf16x6", storage="c128"),
             "bf16x6_c64_f64tol": dict(precision="bf16x6", storage="c64",
                                       jacobi_tol=2048 * 2.0 ** -53),
             "fp64_c128": dict(precision="fp64", storage="c128", svd_precondition=True),
             "fp64_c128_tol30": dict(precision="fp64", storage="c128", svd_precondition=True,
                                     jacobi_tol=2.0 ** -30),
             "fp64_c128_tol27": dict(precision="fp64", storage="c128", svd_precondition=True,
                                     jacobi_tol=2.0 ** -27),
             "bf16x6_c64_local": dict(precision="bf16x6", storage="c64"),
             "fp64_c128_tol30_local": dict(precision="fp64", storage="c128",
                                           svd_precondition=True, jacobi_tol=2.0 ** -30)}
    spec = {k: every[k] for k in args.variants.split(",")}
    hs = {}
    for k, kw in spec.items():
        hs[k] = T.MPS(n, chi, 1e-12, **kw)
        hs[k].copy_from(ref)
    curve = {k: [] for k in spec}
    secs = {k: 0.0 for k in list(spec) + ["pergate_fp64"]}
    for l in range(P, P + K):
        for k in spec:
            if k.endswith("_local"):
                hs[k].copy_from(ref)
        for k in spec:
            t0 = time.perf_counter()
            run_layer_batched(hs[k], layers[l])
            torch.cuda.synchronize()
            secs[k] += time.perf_counter() - t0
        t0 = time.perf_counter()
        run_layer_pergate(ref, layers[l])
        torch.cuda.synchronize()
        secs["pergate_fp64"] += time.perf_counter() - t0
        nr = ref.norm2()
        for k in spec:
            curve[k].append(1.0 - abs(ref.overlap(hs[k])) ** 2 / (nr * hs[k].norm2()))
        log(f"layer {l}: " + ", ".join(f"{k} {curve[k][-1]:.3g}" for k in spec))
    first = next(iter(spec))
    return {"metric": f"1 - F of {first} against the per-gate float64 path after each of {K} "
                      f"layers, chi={chi}",
            "value": curve[first][-1], "unit": "1 - F", "n_gpus": 1, "steps": K,
            "warmup": 0, "ms_per_step": 1e3 * secs[first] / K, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"n=100 benchmark circuit, layers {P}-{P + K - 1} from the "
                                   f"float64 snapshot after {P} layers, chi_max={chi}"},
            "one_minus_F": curve, "seconds": secs,
            "sum_eps_pergate": ref.stats()["sum_eps"]}


def bench_calib(args):
    """Copy kernel of known size, for scaling hardware byte counters: the
    library's storage-conversion kernel (the one tnsim_mps_copy launches) on
    complex128 sites of a synthetic state; each launch on a 1024 x 2 x 1024
    site reads and writes exactly 32 MiB."""
    import torch

    from paper_2601_04422_amd import tnsim as T
    from paper_2601_04422_amd import workloads as W

    n, chi = 24, 1024
    dims = W.saturated_dims(n, chi)
    sites, lams = W.random_canonical_mps(n, dims, 5)
    a = T.MPS(n, chi, precision="fp64", storage="c128", max_layer_gates=1)
    b = T.MPS(n, chi, precision="fp64", storage="c128", max_layer_gates=1)
    a.import_state(sites, lams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.copy_from(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    big = [q for q in range(n) if dims[q] == chi and dims[q + 1] == chi]
    moved = 2 * 16 * sum(dims[q] * 2 * dims[q + 1] for q in range(n))
    return {"metric": "counter calibration: storage-conversion copy of complex128 sites",
            "value": moved / dt / 1e9, "unit": "GB/s", "n_gpus": 1, "steps": 3, "warmup": 0,
            "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "c128", "data": "synthetic",
            "config": {"workload": f"copy of an n={n}, chi={chi} state; sites {big} are "
                                   f"{chi}x2x{chi}: {16 * chi * 2 * chi // 1024} KiB read and "
                                   f"written per launch"}}


def bench_peak(args):
    """Attainable float64 rates of the device: independent chains of the
    matrix-core instruction the contraction kernels use
    (v_mfma_f64_16x16x4f64), of vector FMAs (the pair solve), and of both at
    once (half the wavefronts each), over a grid that fills the chip; best
    of three launches each."""
    from paper_2601_04422_amd import tnsim as T

    m = T.MPS(4, 2, precision="fp64", storage="c128")
    mfma = max(m.probe_fp64("mfma") for _ in range(3))
    valu = max(m.probe_fp64("valu") for _ in range(3))
    mixed = max(m.probe_fp64("mixed") for _ in range(3))
    mfma4 = max(m.probe_fp64("mfma4") for _ in range(3))
    return {"metric": "attainable float64 rate, matrix cores (v_mfma_f64_16x16x4f64 chains)",
            "value": mfma, "unit": "TFLOP/s", "n_gpus": 1, "steps": 3, "warmup": 1,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "8 independent instruction chains per wavefront, 8 "
                                   "workgroups of 4 wavefronts per CU, 2000 x 8 "
                                   "instructions per wavefront"},
            "valu_fma_tflops": valu, "mixed_tflops": mixed, "mfma_4x4x4_tflops": mfma4,
            "published_peak_tflops": FP64_PEAK_TFLOPS}


def main():
    args = parse()
    headline = args.workload == "chi1024"
    if args.precision is None:
        args.precision = "fp64" if headline else "bf16x6"
    if args.storage is None:
        args.storage = "c128" if headline else "c64"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload != "chi1024":
        fn = {"wide": bench_wide, "ansatz": bench_ansatz, "batch": bench_batch,
              "nonlocal": bench_nonlocal, "sample": bench_sample,
              "qasm": bench_qasm, "fidelity": bench_fidelity, "calib": bench_calib,
              "propagate": bench_propagate, "canonical": bench_canonical,
              "peak": bench_peak}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return
    import torch

    from paper_2601_04422_amd import tnsim as T

    n, chi = 100, args.chi
    P, Wu, K = args.prep_layers, args.warmup, args.steps
    KP = K if args.profile_steps < 0 else min(args.profile_steps, K)
    layers = circuit_layers(P + Wu + K)

    # --- preparation (untimed): float64 batched path up to saturation
    ref = T.MPS(n, chi, 1e-12, precision="fp64", storage="c128")
    t0 = time.perf_counter()
    for l in range(P):
        run_layer_batched(ref, layers[l])
        log(f"prep layer {l}: max chi {int(max(ref.bond_dims()))} "
            f"({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0

    # --- batched path from the snapshot, on a stream of its own (the library
    # captures its Jacobi sweeps as HIP graphs there)
    kw = dict(precision=args.precision, storage=args.storage, jacobi_tol=args.jacobi_tol,
              svd_precondition=True)
    stream = torch.cuda.Stream()
    mix = T.MPS(n, chi, 1e-12, stream=stream, **kw)
    tuned = mix.autotune()
    log(f"autotuned launch shapes by pair-count class: rotation rows {tuned[:4]}, "
        f"Gram K-split {tuned[4:]}")
    mix.copy_from(ref)
    for l in range(P, P + Wu):
        run_layer_batched(mix, layers[l])
        log(f"batched warmup layer {l}")
    torch.cuda.synchronize()
    # the same state again, for the profiled pass and the CPU baseline
    snap = T.MPS(n, chi, 1e-12, stream=torch.cuda.Stream(), **kw)
    snap.set_autotune(tuned)
    snap.copy_from(mix)
    gate_inputs = None if args.no_cpu else snapshot_gate(snap, layers[P + Wu], chi)
    full = 0
    total2q = 0
    per_layer = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if not args.circuit:
        for l in range(P + Wu, P + Wu + K):
            tl = time.perf_counter()
            full += count_full(mix, layers[l][2], chi)
            total2q += len(layers[l][2])
            run_layer_batched(mix, layers[l])
            per_layer.append(time.perf_counter() - tl)
            lb = mix.last_batch()
            log(f"batched layer {l}: {per_layer[-1]:.2f} s; sweeps mean {lb[:, 5].mean():.1f}, "
                f"max {lb[:, 5].max()}")
    else:
        # the timed layers as one circuit: gates start when their qubits are
        # free, so the next layer's gates fill the sweeps of the last ones
        circ = [g for l in range(P + Wu, P + Wu + K) for sub in layers[l] for g in sub]
        mix.run_circuit(circ)
        lb = mix.last_batch()
        full = int(np.sum((lb[:, 1] == chi) & (lb[:, 2] == chi) & (lb[:, 3] == chi)))
        total2q = len(lb)
        per_layer.append(time.perf_counter() - t0)
        log(f"batched circuit, layers {P + Wu}-{P + Wu + K - 1}: {per_layer[-1]:.2f} s; "
            f"sweeps mean {lb[:, 5].mean():.1f}")
    torch.cuda.synchronize()
    mix_s = time.perf_counter() - t0
    mix_sweeps = mix.sweep_stats()

    # --- profiled pass: the first KP timed layers again from the same state,
    # every launch bracketed by HIP events on the handle's stream (no graph
    # replay while profiling), for the per-kernel times and the roofline
    snap.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pfull = 0
    if not args.circuit:
        for l in range(P + Wu, P + Wu + KP):
            pfull += count_full(snap, layers[l][2], chi)
            run_layer_batched(snap, layers[l])
    else:
        snap.run_circuit([g for l in range(P + Wu, P + Wu + KP) for sub in layers[l] for g in sub])
    torch.cuda.synchronize()
    prof_s = time.perf_counter() - t0
    prof = snap.profile_read()
    snap.profile(False)
    log(f"profiled pass over {KP} layers: {prof_s:.2f} s")
    same = None
    if KP == K:
        same = 1.0 - abs(mix.overlap(snap)) ** 2 / (mix.norm2() * snap.norm2())
    snap.close()

    # --- per-gate float64 path from the same snapshot, same layers
    pergate = None
    fid_err = None
    if not args.no_pergate:
        for l in range(P, P + Wu):
            run_layer_pergate(ref, layers[l])
            log(f"per-gate warmup layer {l}")
        torch.cuda.synchronize()
        rfull = 0
        t0 = time.perf_counter()
        for l in range(P + Wu, P + Wu + K):
            tl = time.perf_counter()
            rfull += count_full(ref, layers[l][2], chi)
            run_layer_pergate(ref, layers[l])
            log(f"per-gate layer {l}: {time.perf_counter() - tl:.2f} s")
        torch.cuda.synchronize()
        pg_s = time.perf_counter() - t0
        pergate = {"value": rfull / pg_s, "unit": "2q gates/s", "ms_per_step": 1e3 * pg_s / K,
                   "dtype": "f64", "storage": "c128", "svd": "plain one-sided Jacobi on M",
                   "jacobi_sweeps": ref.sweep_stats()}
        ov = ref.overlap(mix)
        fid_err = 1.0 - abs(ov) ** 2 / (ref.norm2() * mix.norm2())

    roof = roofline(prof)
    if roof.get("bound") == "mfma":
        # what the device sustains on the same instruction, measured here
        small = T.MPS(4, 2)
        att = max(small.probe_fp64("mfma") for _ in range(3))
        small.close()
        roof["attainable_mfma_tflops"] = att
        roof["executed_frac_of_attainable"] = roof["executed_frac"] * FP64_PEAK_TFLOPS / att

    cpu = None
    if gate_inputs is not None:
        threads, visible, model = host_cpu()
        log(f"cpu baseline: oracle on one gate, {threads} threads ({model}) ...")
        cpu = cpu_baseline_snapshot(gate_inputs, chi, threads, visible, model)

    value = full / mix_s
    fid_ok = fid_err is not None and fid_err <= FIDELITY_BOUND
    metric = METRIC if (fid_ok or args.no_pergate) else METRIC + " [NOT MET: fidelity bound exceeded]"
    out = {
        "metric": metric,
        "value": value,
        "unit": "2q gates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wu,
        "ms_per_step": 1e3 * mix_s / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"{args.precision} contraction, f64 svd",
        "data": "synthetic",
        "config": {"workload": f"n=100 circuit, layers of Rx,Rz on every qubit then CNOT on "
                               f"alternating bonds; chi_max={chi}, cutoff 1e-12; layers 0-{P-1} "
                               f"untimed (f64), {Wu} warmup + {K} timed layers"
                               + (" (one dependency-scheduled circuit call)" if args.circuit
                                  else " (one call per sublayer)"),
                   "n_qubits": n, "chi_max": chi, "cutoff": 1e-12, "storage": args.storage,
                   "precision": args.precision, "svd": "QR-preconditioned one-sided block Jacobi",
                   "timed_2q_gates": total2q, "autotuned_launch_table": {"rot_rows": tuned[:4], "gram_ksplit": tuned[4:]},
                   "timed_gates_at_full_chi": full, "parallelism": "single gpu"},
        "fidelity_err_vs_fp64": fid_err,
        "fidelity_bound": FIDELITY_BOUND,
        "fidelity_ok": fid_ok if not args.no_pergate else None,
        "all_2q_gates_per_s": total2q / mix_s,
        "pergate_fp64": pergate,
        "speedup_vs_pergate": (value / pergate["value"]) if pergate and pergate["value"] else None,
        "jacobi_sweeps": mix_sweeps,
        "prep_s": prep_s,
        "layer_s": [round(x, 3) for x in per_layer],
        "profiled_pass": {"layers": KP, "s": prof_s,
                          "gates_per_s": pfull / prof_s if pfull else None,
                          "one_minus_F_vs_timed": same},
        "kernel_ms": {k: round(v["ms"], 3) for k, v in prof.items() if v["launches"]},
        "kernel_rates": kernel_rates(prof, args.precision),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
