"""MI355X (gfx950) stochastic-cutoff Monte-Carlo step: switching (Eqs. 1-3),
Kuhn-Wattenhofer colouring (Sec. 2.3) and colour-parallel Metropolis (Fig. 1),
as HIP kernels behind the C-ABI of include/sco.h."""
from .chain import SCO, ChainParams, workspace_size
from ._lib import ScoError, lib

__all__ = ["SCO", "ChainParams", "workspace_size", "ScoError", "lib"]
