"""Copy kernel of known size, for scaling hardware byte counters.

Runs the library's storage-conversion kernel (used by tnsim_mps_copy) on
complex128 sites of a known state: each launch reads and writes exactly
16 * (chiL * 2 * chiR) bytes.  Profilers' FETCH_SIZE / WRITE_SIZE of these
launches divided by those bytes give the counter scale.
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
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
    for _ in range(3):
        b.copy_from(a)
    torch.cuda.synchronize()
    big = [q for q in range(n) if dims[q] == chi and dims[q + 1] == chi]
    print(f"copy kernels: sites {big} have {chi * 2 * chi} complex128 entries "
          f"= {16 * chi * 2 * chi / 1024:.0f} KiB read and written per launch")


if __name__ == "__main__":
    main()
