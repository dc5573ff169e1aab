"""MI355X-native coupled lattice Boltzmann crystal-growth solver (arXiv 2206.02145).

The solver runs in hand-written HIP kernels behind the C-ABI library ``liblbcg.so``; the
``lbcg`` module is its thin ctypes binding. Importing this package loads nothing.
"""
