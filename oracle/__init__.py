"""Plain FP64 CPU oracle of the visual-inertial Gauss-Newton step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP path: it is written from the
paper's definitions (Sec. 3.1: Eq. 1 vision residual, Eq. 2-3 inertial
residual, Eq. 4 Schur-complement step) in NumPy float64, with no blocking or
fusion beyond what those definitions state.

Modules
  so3        rotation exponential/logarithm and right Jacobians
  preint     IMU preintegration (Sec. 3.1 "Inertial Residual", Forster et al.)
  vision     Eq. 1 residual and its analytic Jacobians, per edge
  imu        Eq. 3 residual, its analytic Jacobian, and the factor information
  normal_eq  Eq. 4: blocks B, E, C, w_xi, w_d; damping; Schur elimination
  dense      full stacked-Jacobian normal equations for tiny problems (a pin)
  solve      one step (linearise, eliminate, solve, retract) and the iteration
  cnn        the learned warm-start network (features, forward, backward,
             AdamW), the reference of the warm-start kernels
  gauss      the loop-closure update of a Gaussian map (Sec. 3.3, Eq. 7-8)
  predict    a new keyframe's initial state from preintegration, with the
             covariance-trace fallback (Sec. 3.1, frontend tracking)
  inertial_init  IMU initialisation stage 2, inertial-only optimisation of
             gravity direction, log-scale, velocities and biases (Sec. 3.2)
  pgba       loop-closure pose-graph bundle adjustment in Sim(3) (Sec. 3.1,
             Eq. 5): loop-pair vision terms and relative-pose terms

Parity status per function is listed in each module header.  Every function
here is pinned by a CPU test against something other than itself (closed
forms, finite differences, a dense textbook solve, invariants).
"""
from . import so3, preint, vision, imu, normal_eq, dense, solve, cnn, gauss, predict, inertial_init, pgba  # noqa: F401
