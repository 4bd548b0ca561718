"""Oracle: a plain, slow, complex-FP64 CPU reference of the butterfly-accelerated VIE hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product library never calls it and
shares no code with it (no kernels, headers, helpers, tables or constant
generators); it has its own tree, interpolative decomposition, butterfly apply,
preconditioner and GMRES.

Modules and the passage each follows (Sayed, Liu, Gomez, Yucel, IEEE TAP,
"A Butterfly-Accelerated VIE Solver ..."):

* ``vie``      -- voxel collocation of the VIE, eq. (1)-(2) and (4)-(5) with the
                  Green's function of Section II; dense matrix, direct-sum rows,
                  FFT-convolution exact product, plane-wave excitation (Section IV).
* ``tree``     -- the cluster tree T_H by recursive KD bisection (Section III-A).
* ``idec``     -- the interpolative decomposition of eq. (ID) with Frobenius
                  truncation at a tolerance chi.
* ``butterfly``-- nested-ID butterfly construction, eqs. (ID), (nested_basis),
                  (butterfly_mat), and the HOD-BF partition/apply of Section III-A.
* ``precond``  -- the multiplicative inverse form of Algorithm 1 (Section III-B),
                  with each X_tau computed exactly and then compressed at chi_fact.
* ``gmres``    -- right-preconditioned flexible GMRES(m) and a dense LU solve for
                  the preconditioned system of eq. (precon).

Parity status: every function here is pinned by a ``-m "not gpu"`` test against a
closed form, an independent quadrature, a textbook identity, brute force or an
invariant, except the preconditioner's compressed factors themselves (tolerance-
and sampling-dependent, so only their products are pinned; see ``precond``).
"""
