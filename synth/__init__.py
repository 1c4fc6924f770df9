"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package draws random numbers and lays them out; it holds none of the
DMRG arithmetic.  Both the CPU oracle and the GPU path consume what it makes.
"""
