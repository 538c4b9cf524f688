"""MI355X-native multiresolution-adapted lattice Boltzmann hot path.

The compute path is the HIP library ``libmrlbm.so`` (built from ``csrc/``) behind
the C-ABI declared in ``include/mrlbm.h``; ``mrlbm`` is its thin ctypes binding.
Importing this package loads nothing: the library is loaded on first use, and
its absence is an error.
"""
