"""MI355X-native FFT-based Core-AFD (adaptive Fourier decomposition) maximal-selection loop.

The decomposition runs in hand-written HIP kernels for gfx950 behind the C ABI
of include/afd.h (libafd.so); this package holds the kernels' sources, the
build script and a thin ctypes binding.
"""
from .afd import AfdError, Group, Plan, Result, load_library, workspace_bytes  # noqa: F401

__all__ = ["AfdError", "Group", "Plan", "Result", "load_library", "workspace_bytes"]
