"""MI355X-native streamed GWAS generalized-least-squares solver.

The compute path lives in the HIP library ``libgls.so`` (C-ABI, see
include/gls.h); this package is its thin Python binding plus the seeded
synthetic-input generators.
"""
