"""MI355X (gfx950) library for the clustered spectral likelihood of parametric CMB component
separation (arXiv 2604.08463): segment preparation, SED tables, the fused per-pixel
likelihood + adjoint kernel, compensated per-cluster reductions and a batched projected L-BFGS,
behind the C ABI of ``include/cs.h``.  This package is the thin Python binding.
"""

from ._lib import (  # noqa: F401
    CONVERGED,
    LS_FAIL,
    MAXITER,
    NONFINITE,
    NOT_PD,
    RUNNING,
    SOLVER_ADATOPK,
    SOLVER_LBFGS,
    CsError,
    OptState,
    Problem,
    default_opts,
    item_range,
    kmeans_batch,
    kmeans_batch_static,
    load,
)
from .autograd import CsLikelihood, neg2logl  # noqa: F401
