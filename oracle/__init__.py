"""FP64 CPU oracle of the two-level BPJD method: test infrastructure only.

Imported by the tests, the smoke check and the CPU-baseline leg of the
benchmark; never by the product path.
"""
