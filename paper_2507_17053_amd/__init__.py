"""MI355X-native matrix-free shifted-boundary (SBM) Poisson operator.

The compute path is the HIP library ``libsbm.so`` behind the C ABI in ``include/sbm.h``;
``paper_2507_17053_amd.sbm`` is its thin ctypes binding.  Importing the package does not
load the library: ``from paper_2507_17053_amd import sbm`` does, and fails loudly when it
has not been built.
"""
__all__ = ["sbm", "inputs"]
