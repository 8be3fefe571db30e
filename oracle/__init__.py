"""FP64 CPU oracle for SegSALSA-STR (arXiv 1504.07028): test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package; the HIP library and its binding never do.
"""
