"""MI355X-native parallel Graver-basis extraction (hot path).

The compute path lives in a C-ABI shared library of hand-written HIP
kernels for gfx950 (``csrc/``); ``graver`` is the thin ctypes binding with
the same entry-point names.  ``workloads`` draws seeded synthetic
instances.  Importing the package does not load the library.
"""
