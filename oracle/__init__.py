"""FP64 CPU oracle of the block-based MR Euler solver: test infrastructure only.

Imported by the test suite, the smoke check and the benchmark's CPU-baseline leg; never
by the product path.
"""
