"""CPU oracle for the multi-period AC OPF model evaluation.

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  The product path never imports it.
"""
