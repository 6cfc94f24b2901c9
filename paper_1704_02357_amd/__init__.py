"""MI355X (gfx950) implementation of the spherical-harmonic FFT estimator of galaxy
power-spectrum multipoles with a local line of sight (Hand, Li, Slepian & Seljak 2017).

The numerical work runs in the HIP library ``libpkm.so`` (C ABI in ``include/pkm.h``);
this package only marshals arguments (``pkm.py``) and builds the library (``build.py``).
"""
from .pkm import (  # noqa: F401
    ABI_VERSION, CIC, NGP, TSC, FP32, FP64, SPHERICAL, CARTESIAN, Batch, Plan, PkmError, Server, autotune, lib_path, load_library,
    kaiser_wedge_gamma, nonuniform_mu_edges, plan_footprint, wedges,
)
