"""FP64 CPU oracle for the tokenizer round trip (test infrastructure only).

This package is the plain, slow, obviously correct definition of what the
HIP library computes.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library: the only common dependency is the
seeded input generator in ``synth``, which holds none of the method's
arithmetic.
"""
from .tokenizer import *  # noqa: F401,F403
