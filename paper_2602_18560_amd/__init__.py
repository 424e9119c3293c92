"""gbsub: MI355X-native iterative galactic-binary subtraction.

The HIP library (``libgbsub.so``) is loaded by :mod:`paper_2602_18560_amd.gbsub`
on first use; importing the package itself loads nothing.
"""
__all__ = ["gbsub", "inputs"]
