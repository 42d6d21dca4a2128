"""Plain FP64 CPU oracle for the resistive / two-fluid SRMHD IMEX scheme.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg; never by the product package.
"""
