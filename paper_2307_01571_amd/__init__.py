"""MI355X-native FFT split-operator propagator for the 2D Dirac equation.

The compute path is the C-ABI library ``libqw.so`` (hand-written HIP for
gfx950, declared in ``include/qw.h``); ``paper_2307_01571_amd.qw`` is its thin
ctypes binding.  Importing this package does not load the library.
"""
__all__ = ["qw", "workloads"]
