"""TEST INFRASTRUCTURE -- the oracle package (serial CPU reference of the step).

Only the test suite, __graft_entry__.smoke() and the CPU-baseline leg of
bench.py may import it; the product path never does.
"""
