"""Seeded synthetic LP generators shared by the tests, the benchmark and the
CPU reference.

This package only draws random problem data (a constraint matrix, a planted
primal/dual optimum and the right-hand sides that make it optimal).  It holds
none of the solver's arithmetic: no residuals, no sketch, no factorisation.
"""
from .planted import (  # noqa: F401
    PlantedLP,
    dense_planted,
    csr_planted,
    config_lp,
    batch_lp,
    batch_shape,
    serving_trace,
    serving_lp,
    sketch_seed,
    CONFIGS,
)
from .svm import SvmLP, svm_lp, svm_shape_lp, SVM_SHAPES  # noqa: F401
