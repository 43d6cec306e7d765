"""MI355X-native Monte Carlo collision term for the quark-gluon Boltzmann equation.

The solver lives in the C-ABI library ``libqgbe.so`` (HIP kernels for gfx950);
``paper_1912_04457_amd.qgbe`` is its thin ctypes binding.
"""
