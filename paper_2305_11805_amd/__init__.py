"""MI355X-native mBP descriptor + per-species MLP energy/force path (PANNA 2.0 hot path).

Importing the package loads nothing; the HIP library is opened on first use
by ``paper_2305_11805_amd.nnpot``.
"""
