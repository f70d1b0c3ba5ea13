"""MI355X (gfx950) Galerkin boundary-integral Poisson-Boltzmann operator and
solver: Cartesian Taylor FMM far field, stored Galerkin near field with
singular cubature, block-diagonal preconditioner, GMRES / mixed-precision
flexible GMRES, solvation energy.  The computation lives in libfagbi.so (HIP);
this package only marshals arguments to its C ABI."""
from ._lib import (BASIS_S0, BASIS_S1, FP64, MIXED, MLP_GATED, MLP_OFF, MLP_PRECOND, PART_ALL, PART_FAR, PART_NEAR, PRECOND_BLOCK, PRECOND_GROUP,
                   PRECOND_DIAG, PRECOND_NONE, RADII_CLUSTER, RADII_LEVEL, FagbiError, Handle, default_params,
                   load)

__all__ = ["BASIS_S0", "BASIS_S1", "FP64", "MIXED", "MLP_GATED", "MLP_OFF", "MLP_PRECOND", "PART_ALL", "PART_FAR", "PART_NEAR", "PRECOND_BLOCK", "PRECOND_GROUP",
           "PRECOND_DIAG", "PRECOND_NONE", "RADII_CLUSTER", "RADII_LEVEL", "FagbiError", "Handle", "default_params",
           "load"]
