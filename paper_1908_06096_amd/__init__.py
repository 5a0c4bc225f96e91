"""MI355X-native spherical-harmonic transform (full and octahedral reduced
Gaussian grids) behind a C-ABI library of hand-written HIP kernels.

Importing the package loads nothing; ``paper_1908_06096_amd.sht`` loads the
compiled library and raises if it is missing."""
