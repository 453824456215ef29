"""One small run of the GPU path on cuda:0, checked against the CPU oracle."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run() -> None:
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from oracle import oracle as O
    from paper_2601_04422_amd import tnsim as T
    from paper_2601_04422_amd import workloads as W

    cfg = W.config_small()
    m = T.MPS(cfg.n, cfg.chi_max, cfg.cutoff, device="cuda:0")
    m.run_layers(cfg.layers)
    o = O.OracleMPS(cfg.n, cfg.chi_max, cfg.cutoff)
    o.run_layers(cfg.layers)
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(16):
        bits = rng.integers(0, 2, cfg.n)
        worst = max(worst, abs(m.amplitude(bits) - o.amplitude(bits)))
    if worst > 1e-12:
        raise AssertionError(f"smoke: amplitude mismatch {worst:.3e}")
    if list(m.bond_dims()) != list(o.bond_dims()):
        raise AssertionError("smoke: bond dimensions differ from the oracle")
    print(f"smoke ok: n={cfg.n} 2q gates={cfg.n2q()} max |amp diff|={worst:.2e}")


if __name__ == "__main__":
    run()
