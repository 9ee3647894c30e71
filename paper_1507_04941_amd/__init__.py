"""gsf: MI355X-native hot path of a filter-based HI source finder.

Separable 3-D Gaussian filter bank, per-voxel local mean / standard deviation
and mean + k*std voxel selection (Westerlund & Harris, Eq. 2 and §3.3), as
hand-written HIP kernels for gfx950 behind a C-ABI library (``libgsf.so``,
declared in ``include/gsf.h``).  ``binding`` marshals torch tensors into that
library; ``synth`` makes seeded synthetic input cubes.

Importing the package loads nothing; the library is opened on first use.
"""
