"""hisv: partitioned (Gather-Execute-Scatter) state-vector simulation on MI355X.

The compute path is the native library ``libhisv.so`` (hand-written gfx950
HIP kernels behind a C ABI, declared in ``include/hisv.h``); ``hisv`` is its
thin ctypes binding.  Importing the package does not load the library, so
``workloads`` (the seeded circuit generators) can be used on any machine.
"""

__all__ = ["hisv", "workloads"]
