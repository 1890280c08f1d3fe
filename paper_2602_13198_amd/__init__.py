"""MI355X-native superphoton Monte Carlo radiative transfer (grmonty-style,
after Naethe Motta, Nemmen & Joshi, arXiv 2602.13198).

The hot path runs as hand-written HIP kernels for gfx950 in ``libgm.so``
behind a C ABI (``include/gm.h``).  :mod:`paper_2602_13198_amd.gm` is the
ctypes binding; :mod:`paper_2602_13198_amd.workloads` builds seeded inputs.
Importing this package does not load the GPU library.
"""
__all__ = ["gm", "workloads"]
