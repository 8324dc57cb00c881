"""LBVH geometric search on the AMD MI355X (gfx950).

``paper_1908_11807_amd.abx`` is the Python binding of the C-ABI library
``libabx.so`` (hand-written HIP kernels); ``datagen`` draws the seeded
synthetic inputs.  Importing the package loads nothing: the library is
loaded on first use and a missing library is an error, never a fallback.
"""
