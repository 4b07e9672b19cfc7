"""Aggregated FP64 sub-grid hydro step for MI355X (gfx950).

The compute path is the HIP library ``libhydroagg.so`` built from ``csrc/``
behind the C ABI in ``include/hydroagg.h``; ``hydroagg`` is its thin ctypes
binding.  ``workloads`` draws the seeded synthetic inputs.
"""
