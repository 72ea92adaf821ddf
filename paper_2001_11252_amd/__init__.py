"""MI355X-native resonant-line Monte Carlo transfer (RASCAS method,
Michel-Dansac et al. 2020) behind the C ABI of ``include/rmc.h``.

Importing the package loads nothing native; ``paper_2001_11252_amd.rmc``
loads ``librmc.so`` and fails loudly if it is missing.
"""
__all__ = ["workloads"]
