"""CPU reference (oracle) for the electron Monte Carlo hot path.

Test infrastructure only: importable from the test suite, the smoke check and
the benchmark's CPU-baseline leg, never from the GPU product path.
"""
