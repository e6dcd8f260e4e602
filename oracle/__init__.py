"""CPU oracle for the least-k search of Erdos' squarefree + power-of-two
conjecture (Hercher, arXiv 2411.01964).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It
shares no code with the GPU library in ``paper_2411_01964_amd``; it is a thin
ctypes wrapper around ``esq_oracle.c`` (plain trial division by odd prime
squares, straight from the definition in Section 2 and Algorithm 2).

Functions whose results are not pinned by anything outside the oracle: none
(see ``tests/test_oracle_pins.py``).
"""
from .oracle import (  # noqa: F401
    build,
    is_squarefree_many,
    mink,
    mink_many,
    nprimes,
    sieve_bits,
    verify_range,
)
