"""MI355X-native hot path of generalized-loss CP tensor completion.

The compute runs in hand-written HIP kernels for gfx950 inside ``libtt.so``,
reached through a C ABI (``include/tt.h``).  ``paper_1910_02371_amd.tt`` is a
thin ctypes binding with the same entry-point names; it raises if the library
is not built.  ``workloads`` synthesizes seeded inputs.
"""
__all__ = ["tt", "workloads"]
