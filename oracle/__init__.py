"""FP64 CPU oracle of the spherical-harmonic transform (test infrastructure
only: used by the tests, the smoke check and the benchmark's CPU baseline,
never by the product path)."""

from . import vector_oracle  # noqa: F401
from .sht_oracle import (  # noqa: F401
    dft_analysis,
    dft_synthesis,
    direct,
    gauss_newton,
    grid_geometry,
    inverse,
    nspec_of,
    pbar,
    spec_index,
)
