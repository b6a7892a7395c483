"""Seeded synthetic inputs for the LDPC decoder: codes, codewords, channel LLRs.

Shared by the tests, the benchmark and the oracle's callers.  It contains no
step of the decoding method itself.
"""
from . import channel, codes, configs, gf2  # noqa: F401
