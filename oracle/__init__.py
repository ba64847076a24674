"""Plain FP64 CPU oracle for the implicit-Euler time-periodic problem.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it. It shares no code with the GPU path (no DFT, no Krylov method,
no multigrid); its only common dependency is the seeded problem descriptions in
``workloads``.

What it computes (all in float64, numpy + scipy.sparse):

* ``fem``       P1 finite elements on the uniform grid: stiffness S, sigma-weighted
                consistent mass M, load b, the nonlinear operator K(u) and its
                Jacobian, and the energy whose gradient K is (Sec. 4, test problem).
* ``periodic``  the space-time operator A(U)^n = M d_tau u^n + K(u^n) with
                u^0 = u^N (Problem 1, eqs. (disc1)-(disc2)), the residual F - A(U),
                the fixed-point iteration (eqs. (iter1)-(iter2)) with
                Khat = nu_max * S and an exact inner periodic solve by sparse LU of
                the assembled space-time matrix (oracle A) or of the 2-D matrix
                M/tau + Khat with period sweeps (oracle B), an all-at-once Newton
                solve (method (M2) without multigrid in time) and sequential
                nonlinear time stepping (method (M3)).
* ``adjoint``   the cycle-averaged eddy-current loss tau sum_n d u^T M d u, the
                Jacobian dA/dU, the adjoint state of the transposed (backward in
                time, periodic) linearised system by sparse LU, and the gradients of
                the loss with respect to the per-triangle nu scale and conductivity.

Where the paper leaves a convention open, the docstring of the function that uses it
states the reading taken.
"""
from . import adjoint, fem, periodic  # noqa: F401
