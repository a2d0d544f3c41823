"""FP64 CPU oracle of the multi-implicit SDC schemes of Hamon, Day & Minion
(arXiv:1801.01201): serial MISDC, MISDCQ, the concurrent CISDCQ-nu scheme and
the fully coupled IMEXQ comparison scheme.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the GPU library and never reads any of its results.

Modules
-------
coefficients  Gauss-Lobatto nodes, the integration matrix Q, the implicit
              weights (backward-Euler and LU trick) and explicit weights.
sdc           The generic step/sweep drivers of every scheme, written term by
              term in the order of the paper's update equations.
linear        The scalar linear model problem, its iteration matrix and the
              cost ratio R_nu.
chemistry     Mass-action kinetics, thermodynamics and the per-cell
              backward-Euler reaction solve (Newton, analytic Jacobian).
transport     Periodic finite-volume advection and diffusion operators and the
              implicit diffusion (Helmholtz) solves, done by a direct solver.
adr           The advection-diffusion-reaction flame problem that ties the
              chemistry and transport together for the SDC drivers.
collocation   Brute-force solution of the collocation system (the fixed point
              of every sweep).
nagumo        The paper's 1-D nonlinear test problem.
mlp           The dense network of the learned Newton guess: forward pass,
              mean-squared-error gradients, Adam, bfloat16 rounding.
"""
