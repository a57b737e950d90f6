"""CPU oracle for star-stencil sweeps (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg import it.
"""
