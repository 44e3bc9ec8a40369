"""Seeded, synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds parameter sets (explicit prime chains), the synthetic
network descriptions and the seeded input arrays.  It contains none of the
homomorphic arithmetic: no NTT, no key switching, no encoding.  Both the CPU
oracle and the GPU library receive what is generated here as plain inputs.
"""
