"""CT-AUX walker for AMD MI355X: HIP kernels behind a C ABI (include/dcax.h).

``paper_1901_01047_amd.dcax`` is the Python binding; ``build`` compiles the
shared library in-tree.
"""
