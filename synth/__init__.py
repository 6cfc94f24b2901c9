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
    modulated_box,
    uniform_survey_randoms,
    config_c1,
    config_c2,
    config_c3,
    batch_mock,
)


def catalog_digest(*catalogs) -> str:
    """Short SHA-256 of the positions, weights and densities of the given catalogs, used to
    check that a regenerated seeded catalog is the one a stored result was computed for."""
    import hashlib

    import numpy as np

    h = hashlib.sha256()
    for c in catalogs:
        for a in (c.pos, c.w, c.nbar):
            if a is not None:
                h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()[:16]
