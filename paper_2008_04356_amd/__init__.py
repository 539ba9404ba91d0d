"""MI355X-native sliding-mesh mortar interface operator (arXiv 2008.04356).

The operator lives in the HIP library ``libmortar.so`` (C ABI declared in
``include/mortar.h``); :mod:`paper_2008_04356_amd.mortar` is its thin ctypes binding and
:mod:`paper_2008_04356_amd.workloads` generates seeded synthetic face data.
"""
__all__ = ["mortar", "workloads"]
