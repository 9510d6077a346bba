"""FP64 CPU oracle of the PUSCH receive chain (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package; the HIP product path never does.
"""
