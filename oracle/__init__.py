"""FP64 CPU oracle for exact Gaussian-process training (BBMM), test infrastructure only.

This package is the plain, slow, obviously correct reference that the GPU
library is checked against.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the library itself never does,
and the oracle never imports the library.  The two share no code: the only
arrays they both see come from the seeded generators in ``synth``.

Modules and what they follow (Sun, Cheng & Miller, "Molecular Energy Learning
Using Alternative Blackbox Matrix-Matrix Multiplication Algorithm for Exact
Gaussian Process"):

* ``kernel``   Matern-5/2 / RBF ARD kernel and K_hat = K + sigma^2 I
               (Sec. 2.2 below Eq. 1; Matern-5/2 named in Sec. 4).
* ``exact``    dense Cholesky solve, log-det, log marginal likelihood (Eq. 2),
               its analytic gradient and the predictive mean/variance (Eq. 1).
* ``pivchol``  pivoted-Cholesky preconditioner P = L L^T + sigma^2 I (Sec. 3.2).
* ``probes``   SplitMix64 Rademacher probes, preconditioned as b = L e1 + sigma e2
               (Sec. 3.1, right-hand sides of block CG).
* ``mbcg``     textbook modified batched preconditioned CG with Lanczos
               tridiagonals, stochastic Lanczos quadrature and trace estimates
               (Sec. 3.1-3.2; mBCG of Gardner et al. 2018 as the paper uses it).
* ``altbbmm``  block CG with a shared block Krylov space (Sec. 3.1) and the
               symmetric Nystrom preconditioner of AltBBMM (Sec. 3.2).
* ``lanczos``  Lanczos variance cache for fast predictive variances.
* ``gradient`` the bilinear forms sum_c w_c u_c^T (dK_hat/dtheta) w_c.

Everything is FP64 numpy/scipy.  Pins (independent checks of this oracle) are
in ``tests/test_oracle_*.py``.
"""
