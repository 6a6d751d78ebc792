"""FP64 CPU oracle for the two-fluid SPH / IDIC step -- test infrastructure only.

Importable only from the test suite, the smoke check and the benchmark's
CPU-baseline leg.  It shares no code with the HIP library.
"""
