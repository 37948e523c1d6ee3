"""Plain FP64 CPU oracle for the parallel orbital-updating (ParO) method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP path.

Contents (each function cites the passage of Dai, Gong, Zhou and Zhu,
"A parallel orbital-updating approach for electronic structure
calculations", arXiv:1405.0260, that it follows):

  fem        P1 finite elements on a Kuhn-tetrahedral box mesh: the bilinear
             form a(u, v) = 1/2 (grad u, grad v) + (V u, v) and the L2 inner
             product (Sec. 2 preliminaries; eq. (eq-operator-A); Appendix,
             the linear operator L and its form a(., .)).
  paro       Algorithm A.1 / Algorithm 3.2 (Steps 1, 3, 4) with Jacobi-PCG
             source solves and a Rayleigh-Ritz projection.
  reference  The plain definition of the ParO fixed point: the lowest N
             eigenpairs of the discrete problem (eq. (fem-eigen)) from
             library eigensolvers.
  kohn_sham  Density, Hartree (Poisson) and Slater-exchange potentials for a
             self-consistent ParO (Sec. 2 Kohn-Sham equation; Algorithm 3.1).
  nonlocal_  The nonlocal pseudopotential term V_nl u = sum_j (u, zeta_j)
             zeta_j as the rank-k Galerkin operator Z Z^T (Sec. 2).
  adapt      Step 2 of Algorithm 3.1: residual estimator, Doerfler and
             maximum marking (Sec. 2 adaptive finite element approximation,
             eqs. (dorfler-strategy), (maximum-strategy)), conforming
             bisection, P1 transfer of the orbitals, and the ParO loop with
             an adaptive Step 2.
"""
