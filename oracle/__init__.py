"""FP64 CPU oracle for convolutional gridding and degridding.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, link or call
anything in this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the HIP library.
"""
from .oracle import *  # noqa: F401,F403
