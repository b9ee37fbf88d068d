"""MI355X library for advancing stiff parabolic operators (anisotropic Spitzer
conduction, artificial viscosity) by RKL2 super time-stepping or backward
Euler + PCG, after Caplan, Mikic, Linker & Lionello (2016).

The compute path is the HIP library libsts.so (C ABI in include/sts.h);
this package is its thin Python binding.  Importing it does not load the
library; the first call (or ``load()``) does, and fails loudly if the library
has not been built (``python -m paper_1610_01265_amd.build``).
"""
from ._binding import (  # noqa: F401
    BC_DIRICHLET,
    BC_PERIODIC,
    BC_ZEROFLUX,
    CARTESIAN,
    LIB_PATH,
    PC_BLOCK_ILU0,
    PC_JACOBI,
    SHELL_BC,
    SPHERICAL,
    STS_BREAKDOWN,
    STS_EINVAL,
    STS_NOT_CONVERGED,
    STS_OK,
    Context,
    StsError,
    apply_F,
    be_pcg_solve,
    exported_symbols,
    load,
    rkl2_step,
    sts_be_residual,
    sts_create,
    sts_destroy,
    sts_dt_euler,
    sts_set_dirichlet,
    sts_set_isotropic,
    sts_set_isotropic_f32,
    sts_set_spitzer,
    sts_set_spitzer_f32,
)
