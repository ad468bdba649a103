"""FP64 CPU oracle for the XM hot path (scaled bundle adjustment, arXiv 2502.04640).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything in this package: only the test suite, the smoke check of the
entry module and the CPU-baseline leg of the benchmark use it.  It shares no
code with the HIP library; both read their inputs from the ``scenes`` module.

Everything here is plain numpy/scipy in float64 and follows the paper's
definitions and algorithms in their own order:

* data_matrix  -- Q of Prop. "Scaled-Rotation-Only Formulation" (App. A), two
                  ways: the paper's A-formula and block elimination of the same
                  matrices; the translation/landmark recovery of eq. tpstar.
* manifold     -- cost tr(Q U^T U), Riemannian gradient/Hessian and retraction
                  on the product manifold of Prop. "BM Riemannian Optimization".
* rtr          -- Riemannian trust region with truncated CG (the local
                  optimizer that Section "C++/CUDA-based Riemannian
                  Optimization" defers to Absil et al. 2008 / Boumal 2023).
* certificate  -- dual variable of eq. bm_first_order_optimality, Z(y) of
                  eq. Zofy, minimum eigenvalue, suboptimality eq. suboptimality.
* staircase    -- Algorithm "Riemannian Staircase".
* rounding     -- top-3 eigenvectors of X, projection to scaled rotations,
                  anchoring (Prop. "SDP Relaxation" and the text after it).
* adjoint      -- gradients of the optimum w.r.t. the lifted keypoints and
                  weights (envelope theorem + implicit function theorem).

Parity status of each function is stated in its docstring; every function is
pinned by a test in tests/test_oracle_*.py against something other than itself.
"""
