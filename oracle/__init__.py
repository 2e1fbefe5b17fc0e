"""CPU oracle for bound propagation and probing (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product path (``paper_2510_20499_amd``) never does.
"""
from .oracle import (  # noqa: F401
    BP_INFEASIBLE, BP_OK, BP_ROUND_LIMIT, MODE_DEFINITION, MODE_WORKLIST, Options,
    bind, build, compile_to, exact_sum, load, probe, probe_box, probe_order, propagate, repair, round_,
    scores,
    validate,
)
