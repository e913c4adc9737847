"""CPU oracle (test infrastructure only).

A plain, slow FP64 implementation of what the GPU library computes, written
from the paper's definitions.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and the
two share no code.  See ``oracle.mpdist`` for the definitions followed.
"""
from .mpdist import *  # noqa: F401,F403
