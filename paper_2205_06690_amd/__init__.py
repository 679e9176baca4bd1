"""MI355X-native stochastic-W Bethe-Salpeter hot path.

Importing the package loads nothing native; ``paper_2205_06690_amd.bse``
binds the HIP library and raises if it is missing.
"""
__all__ = ["inputs", "bse"]
