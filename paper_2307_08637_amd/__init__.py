"""Learned sample sort for AMD MI355X (gfx950).

The sort runs entirely in hand-written HIP kernels behind a C ABI
(``include/lsort.h``, built into ``liblsort.so`` next to this file).  The
Python layer in :mod:`paper_2307_08637_amd.lsort` only marshals torch device
tensors and streams to that ABI; :mod:`paper_2307_08637_amd.inputs` holds the
seeded synthetic workloads.  Import the submodules explicitly.
"""
