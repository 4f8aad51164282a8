"""Plain CPU oracle of SPHINCS+ signing (SHA2 "simple"), for tests only.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The GPU library never calls
it: it shares no code with ``paper_2512_23969_amd``.

The arithmetic lives in ``slh_oracle.c`` (plain C, one function per
definition of FIPS 205 / FIPS 180-4 / FIPS 198-1 / RFC 8017); this module is
a ctypes wrapper around the shared library built from it.
"""
from .oracle import *  # noqa: F401,F403
