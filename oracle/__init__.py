"""FP64 CPU oracle for PSCA detection: test infrastructure only.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The HIP library never calls it.
"""
from .psca_oracle import *  # noqa: F401,F403
from .psca_oracle import (ML_K, MAP_K, ML_UD, MAP_UR, MAP_K2, VARIANT_NAMES, Problem,  # noqa: F401
                          AREA_UNIFORM, UNIFORM_IN_D,
                          PowerLawPrior, make_prior, psca, psca_iteration, step_sizes,
                          problem_from_instance, sample_covariance, model_covariance,
                          frobenius_inverse, quadratic_forms, objective, equal_error_rate)
