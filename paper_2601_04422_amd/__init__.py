"""MPS gate application on MI355X (gfx950): Python binding of the tnsim C ABI.

The compute path lives in the HIP shared library built from ``csrc/``; this
package only marshals arguments (see ``tnsim.py``).  ``workloads`` holds the
seeded input generators.
"""
__all__ = ["tnsim", "workloads"]
