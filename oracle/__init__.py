"""CPU oracle for the leveled RNS-CKKS CNN evaluator.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import anything under this package; the
product library neither imports nor links it.
"""
