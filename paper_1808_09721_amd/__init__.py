"""MI355X-native (gfx950, HIP, FP64) resistive and two-fluid SRMHD IMEX hot path.

Importing the package loads nothing native; ``paper_1808_09721_amd.rmhd`` holds the
binding to the C-ABI library ``librmhd.so``.
"""
