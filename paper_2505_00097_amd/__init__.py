"""MI355X-native BSSN evolution core (arXiv:2505.00097 hot path).

The compute path is the HIP library libbhah.so (C ABI in include/bhah.h);
`paper_2505_00097_amd.capi` is its thin Python binding. Importing this package
loads nothing; the binding loads the library on first use and raises if it
has not been built.
"""
