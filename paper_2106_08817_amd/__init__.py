"""MI355X (gfx950) semi-Lagrangian geodesic shooting for Metamorphosis / LDDMM
image registration (arXiv:2106.08817): batched forward shooting, cost and a
hand-written discrete adjoint (dH/dp0) behind a C ABI (include/shoot.h)."""
from .api import (  # noqa: F401
    SHOOT_CHECK_FINITE,
    SHOOT_FORCE_GLOBAL_SCATTER,
    SHOOT_FULL_STORE,
    SHOOT_LANES,
    SHOOT_NO_GRAPH,
    SHOOT_SCHEME_EULERIAN,
    SHOOT_SCHEME_MIXED,
    SHOOT_UNFUSED,
    LBFGS,
    PairSpec,
    Plan,
    ShootCost,
    gradient_descent,
    lbfgs,
    shoot_cost,
)
from ._lib import ShootError, load  # noqa: F401
