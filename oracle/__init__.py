"""CPU oracle for the Faddeev-Merkuriev spline-collocation system.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute this package; only the
tests, the smoke check and the benchmark's CPU-baseline leg use it.

The oracle is a plain, slow, FP64 NumPy/SciPy implementation written from the
paper (Gradusov, Roudnev, Yarevsky, Yakovlev, arXiv:2005.05398):

  basis.py     1D Hermite spline bases, node maps, Gauss collocation points
               (Sec. 3.1 local basis, Sec. 4 quintic Hermite S_5^3 + Gauss points)
  physics.py   masses, Jacobi rotation, Coulomb potentials, Merkuriev split
               (Sec. 2.1 eqs. (JacobiTrans), (split3b), (Mcutoff0); Sec. 2.2 X_beta(X_alpha))
  wigner.py    Wigner d / parity-adapted F functions for L > 0 (Sec. 2.2)
  assemble.py  explicit collocation matrix H - E S of eq. (FM-pre) and the
               separable left-hand block L_alpha of eq. (FM-fin) (Sec. 3.1-3.2)
  solve.py     LU solves and residuals
  eigen.py     the mass matrix S and bound-state energies of H c = E S c
               (shift-invert ARPACK, dense QZ for tiny problems)
  symmetry.py  the exchange-reduced equations of two identical particles
               (Sec. 2, eq. (2-sym-part))
  precond_v2.py  the coupled L > 0 preconditioner: the approximate matrix
               script-L of Sec. 3.2 (eq. (prop-eq)) and the Appendix functions g

It shares no code with the HIP path.  Its inputs (problem descriptions, seeded
right-hand sides) come from a data-only module.
"""
