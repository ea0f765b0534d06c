"""MI355X-native Monte Carlo of the 3d Heisenberg spin glass with random
anisotropic couplings (arXiv:1309.1599): checkerboard heat-bath and
overrelaxation sweeps, parallel tempering and FP64 overlap / chirality /
energy reductions in hand-written gfx950 kernels behind a C ABI
(include/ptsg.h).

`ptsg` is the binding of that ABI; `inputs` draws the seeded synthetic
couplings and temperature grids.  Importing the package loads nothing; the
library is loaded on first use and must be built (`python -m
paper_1309_1599_amd.build`).
"""
from . import inputs  # noqa: F401
