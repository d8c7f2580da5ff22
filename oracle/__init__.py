"""CPU FP64 reference (oracle) for the bundle-adjustment hot path.

Test infrastructure only: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.
"""
