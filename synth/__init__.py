"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This package holds random-field and right-hand-side generators only.  It contains
none of the method's arithmetic (no operator, no transform, no solver), so that
the GPU path and the CPU oracle can both draw identical inputs from it without
sharing any computational code.
"""

from .inputs import (  # noqa: F401
    gaussian_random_field,
    lognormal_kappa,
    drifting_kappa_blocks,
    first_block_rhs,
    random_block_vector,
    batched_problem_specs,
)
