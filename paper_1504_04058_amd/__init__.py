"""Additive sweeping preconditioner for the PML-truncated Helmholtz equation
(Liu & Ying) on AMD MI355X: a HIP library with a C ABI (include/asp.h) and a thin
Python binding (``paper_1504_04058_amd.asp``).

Importing the package loads nothing; ``from paper_1504_04058_amd import asp``
loads torch and then libasp.so (built by ``python -m paper_1504_04058_amd.build``).
"""
