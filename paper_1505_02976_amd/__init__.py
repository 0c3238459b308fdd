"""MI355X implementation of the modified lattice-BGK model for convection heat transfer in
porous media at the REV scale (Wang, Mi & Guo, arXiv:1505.02976).

The compute path is the HIP library liblbm.so (C interface in include/lbm.h);
``paper_1505_02976_amd.lbm`` is its Python binding.
"""
from . import lbm  # noqa: F401
from .lbm import Adjoint, Batch, Sim, derived, nusselt_of_porosity, workspace_bytes  # noqa: F401
