"""Primal-dual parallel Gibbs sampling for discrete pairwise MRFs on MI355X.

``paper_1611_06684_amd.pdg`` is the ctypes binding of the C-ABI library
``libpdg.so`` (HIP kernels for gfx950); ``workloads`` holds the seeded
synthetic input generators.
"""
