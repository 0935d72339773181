"""CPU oracle for exact (l,d) planted motif search.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU path (see ``pms_oracle.c`` for what each function follows).
"""
from .oracle import (  # noqa: F401
    OracleError,
    build,
    cd,
    encode,
    hd,
    library_path,
    neighbourhood,
    solve_a,
    solve_b,
    theorem1,
)
