"""CPU oracle for the Kryging hot path (Majumder, Guan, Reich & Saibaba,
"Kryging: Geostatistical analysis of large-scale datasets using Krylov
subspace methods").

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, FP64 reference
that the HIP library is checked against.  Only the test-suite, the smoke
check in ``__graft_entry__.smoke`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The library under ``paper_2012_13133_amd`` never
imports, links or calls anything here, and nothing here imports the library:
the two share no kernels, helpers, tables or constants.

Every function states the passage of the paper it follows.  Where the method
reaches exactly (up to rounding) a result with a plain definition -- the
masked covariance product, the Gaussian log-likelihood, the kriging mean and
variance -- the oracle is that definition written out densely.  Where the
method is an iteration (Lanczos quadrature, conjugate gradients, generalized
Golub-Kahan bidiagonalization, the parametric bootstrap) the oracle takes the
algorithm's steps in the paper's order and notation.

Modules
-------
philox      counter-based RNG (Philox4x32-10) shared by definition with the
            device, Rademacher probes and Box-Muller normals
matern      Matern correlation (Sec. 2) and the anisotropic lag distance
geometry    cell coordinates, lag tables, circulant-embedding lag grid
direct      direct O(p^2) masked covariance product
dense       dense Cholesky log-likelihood and kriging, with covariates (GLS)
lanczos     stochastic Lanczos quadrature for log det (Sec. 3.3 alternative)
cg          textbook conjugate gradients
gengk       generalized Golub-Kahan bidiagonalization (Algorithm 1), low-rank
            posterior variance
sampler     Cholesky and circulant-embedding Gaussian field samplers
bootstrap   parametric bootstrap prediction variance and parameter estimates
            (Sec. 3.5)
fit         profile-likelihood maximisation over (range, nugget ratio)
irregular   Wendland mapping of irregularly spaced observations (Sec. 2)
plik        the paper's own profile likelihood (exact and approximate), the
            quadrant log-determinant, the approximate gradient and the
            rank-one-Hessian trust-region fit

Parity unpinned: none.  Every function has at least one test in
``tests/test_oracle_*.py`` that checks it against something other than
itself (closed forms, library routines, brute force, invariants).
"""
