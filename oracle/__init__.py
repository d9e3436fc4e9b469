"""FP64 CPU oracle of the scale-aware 2D Gaussian rasterizer.

Test infrastructure only: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the product package.
"""
