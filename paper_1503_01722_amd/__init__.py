"""MI355X-native coupled photon-electron Monte Carlo dose engine (the hot path of
arXiv 1503.01722, oclMC), behind the C ABI declared in include/omc.h.

Importing the package loads nothing heavy; ``paper_1503_01722_amd.omc`` holds the
binding to the HIP library and ``paper_1503_01722_amd.workloads`` the seeded
input generators.
"""
__all__ = ["omc", "workloads"]
