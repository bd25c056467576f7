"""CPU float64 oracle of semi-Lagrangian Metamorphosis / LDDMM shooting.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path. It shares no code
with the HIP library.

Parity status of each function (what pins it; tests/test_oracle_*.py):

* gaussian_taps, conv_axis, smooth: SciPy ``correlate1d(mode='constant')``,
  constant preservation away from edges, self-adjointness.
* diff, diff_T: exactness on affine fields, dot-product transpose test,
  closed-form boundary rows.
* feet, interp, interp_grad, interp_T: SciPy ``map_coordinates(order=1,
  mode='nearest')``, torch ``grid_sample(border, align_corners=True)``,
  exact integer shifts, affine reproduction, dot-product transpose test,
  central finite differences of interp.
* step_given_v, step, shoot: identity at zero momentum, constant-image
  invariants, maximum principle at rho = 0, exact integer shift, the sign of
  the transport for a ramp, the constant-image closed form at T = 1.
* cost_terms, cost_and_grad, step_adjoint: closed form at T = 1, central
  finite differences on 16x16 (and 3-D) inputs, autograd of an independent
  torch float64 program.
* deformation: identity at zero momentum, the clamped foot in closed form at
  T = 1, a component that stays the identity when nothing moves along its
  axis, values within the grid.
* step_eulerian_given_v, step_mixed_given_v, shoot(scheme=...): identity at
  zero momentum, exact transport of affine fields by a constant velocity in
  the interior, first-order convergence of the Eulerian time stepping, and
  the stability behaviour the paper reports (Eulerian ripples and failure
  where the semi-Lagrangian scheme keeps the image in range).
* energy: a constant image (only rho ||z||^2 is left) and a unit impulse of
  z on a ramp image (the product of the Gaussian's centre taps), closed forms.
* gradient_descent: the closed form of descent on the quadratic cost of a
  constant source at T = 1 (iterates, costs and every step halving). The
  halving rule (halve the step when the cost at the current iterate exceeds
  the previous one) is this library's convention; the paper names none.
* lbfgs (oracle/lbfgs.py): two-loop recursion against the explicit BFGS
  inverse-Hessian product; convergence on a strictly convex quadratic.
"""
from .shooting import (  # noqa: F401
    Feet,
    Trajectory,
    conv_axis,
    cost,
    cost_and_grad,
    cost_terms,
    deformation,
    diff,
    diff_T,
    divergence,
    energy,
    feet,
    gaussian_taps,
    gradient_descent,
    grid_coords,
    interp,
    interp_T,
    interp_grad,
    max_displacement,
    momentum_field,
    shoot,
    smooth,
    step,
    step_adjoint,
    step_eulerian_given_v,
    step_given_v,
    step_mixed_given_v,
    velocity,
)
from .lbfgs import lbfgs, minimize as lbfgs_minimize, two_loop  # noqa: F401,E402
