"""Seeded synthetic inputs: random lattice circuits, their tensor networks, paths and slices.

Shared by the oracle tests and the GPU path; holds no contraction arithmetic.
"""
