"""MI355X-native Minimod acoustic_iso_cd propagator.

The compute path is the C-ABI library `libminimod.so` (hand-written HIP for
gfx950) declared in `include/minimod.h`; `paper_2007_06048_amd.minimod` is the
thin ctypes binding over it and `paper_2007_06048_amd.workloads` builds seeded
synthetic inputs.  Importing this package loads nothing; the binding loads
the library on first use and raises if it is missing.
"""
