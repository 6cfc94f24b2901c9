"""Seeded synthetic inputs shared by the GPU path's tests/bench and by the oracle.

This package only draws random catalogs (positions, weights, number densities).
It holds none of the estimator's arithmetic: no painting, no Fourier transform of
the galaxy field, no spherical harmonics, no binning.
"""
from .lognormal import (  # noqa: F401
    Catalog,
    SurveyGeometry,
    lognormal_survey,
    uniform_box,
    uniform_survey_randoms,
    config_c1,
    config_c2,
    config_c3,
    batch_mock,
)
