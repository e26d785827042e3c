"""CPU oracle for the PRAND generators -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  It wraps ``liboracle.so``, built from
``prand_oracle.c`` (plain C, exact integer arithmetic), which shares no code
with the GPU library.
"""
from .oracle import Oracle, build_oracle, ORACLE_SO  # noqa: F401
