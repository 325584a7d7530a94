"""MI355X-native ESCG Monte Carlo hot path (arxiv 2508.16639).

The compute path is a HIP shared library (``csrc/``, built for gfx950) with a
C ABI declared in ``include/escg.h``.  ``escg.py`` marshals arguments to it;
``workloads.py`` describes the synthetic inputs.  Importing this package does
not load the library: ``escg.lib()`` does, and raises if it was not built.
"""
__all__ = ["escg", "workloads"]
