"""CPU FP64 oracle for the Wilson-Dirac / CG / HMC hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.
"""
