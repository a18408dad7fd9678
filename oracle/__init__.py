"""FP64 CPU oracle of the moving-boundary cut-cell split step (arXiv:1711.11361).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU-baseline leg of
bench.py.  The product package never imports anything from here.
"""
