"""FP64 CPU oracle for the VGF / Hockney-Eastwood free-space Poisson solves.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it. The GPU library neither imports nor links it, and it
shares no code with the GPU path. See vgf_oracle.c for the definitions and
their citations (arXiv:2103.08531, Secs. I-III).
"""
from .oracle import *  # noqa: F401,F403
