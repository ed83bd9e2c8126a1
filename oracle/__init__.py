"""FP64 CPU oracle of the AP-Cloud field solve -- test infrastructure only.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library.
"""
from .oracle import (OracleCloud, build_oracle_lib, wls_fit, monomials, thresholds,
                     num_unknowns, push)

__all__ = ["OracleCloud", "build_oracle_lib", "wls_fit", "monomials", "thresholds",
           "num_unknowns", "push"]
