"""FP64 CPU oracle for the per-vertex reaction + SDC stage.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or executes this package; only the test suite,
the smoke check and the CPU-baseline leg of the benchmark call it.

What it computes (paper section 3.3.2, equations genODE, picard_form,
residual, sdc_ode and sdc): for every vertex the state X = (v, w, c) obeys
dX/dt = F(X) with the diffusion term held fixed; one time step runs a
backward-Euler local-Newton predictor over the Gauss-Lobatto sub-intervals and
then K linearised implicit SDC sweeps.  The implementation is deliberately
plain: numpy arrays vectorised over vertices, fp64 throughout, the Jacobian
from forward-mode dual numbers (exact derivatives, as the paper requires for
its Rosenbrock and SDC systems) and a dense pivoted LU (LAPACK via
numpy.linalg.solve) in place of the GPU's static sparse elimination.

Modules:
  ad        forward-mode dual numbers over numpy arrays
  lr91      Luo-Rudy 1991 ventricular model (8 states)
  tt06      ten Tusscher-Panfilov 2006 epicardial model (19 states)
  testmodels  scalar linear / logistic problems with closed forms
  models    registry
  lobatto   Gauss-Lobatto nodes and the spectral integration matrix S
  sdc       predictor + sweeps + time loop
  rest      resting state F(X*) = 0
  opcount   algorithmic operation counts per vertex-step
"""
