"""MI355X-native moving-boundary cut-cell split solver (arXiv:1711.11361).

The numerical hot path lives in the HIP library ``libcutcell.so`` (C ABI declared in
``include/cc.h``); :mod:`paper_1711_11361_amd.cc` is its thin ctypes binding and
:mod:`paper_1711_11361_amd.workloads` builds the seeded synthetic inputs.
"""
