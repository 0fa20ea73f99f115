"""FP64 CPU oracle of the localized sparsifying preconditioner.

Test infrastructure only: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the HIP library never does.
"""
