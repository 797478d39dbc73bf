"""CPU FP64 oracle for the linearized VHS collision operator.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import anything from this package.
The GPU library never calls it, links it or falls back to it, and this
package imports nothing from the GPU library.

Reference: Yin, Cai, Wang, "A fast Fourier spectral method for the
linearized Boltzmann collision operator" (arXiv 2503.09580).

Modules
-------
quadrature   Gauss-Jacobi-Radau rule in the relative speed g (Sec. 2.3,
             eq. (13); Sec. 4.1) and the hemisphere product rule used by
             the binary method.
grid         Collocation grid, index sets and dense DFT matrices (Sec. 2.3).
fast_direct  O1: the fast linearized method (Sec. 3.2, eqs. (20), (23),
             (24); Algorithm 1) evaluated with dense DFT matrices and the
             naive (direct-sum) cyclic convolution for psi_j.
alg1         Algorithm 1 step by step with a library FFT as the transform
             primitive (used as the CPU throughput baseline).
binary       O2: the binary-operator spectral method (Sec. 2.3, eq. (14))
             with an explicit hemisphere quadrature, evaluated for
             L_bin[h] = Q(M,h) + Q(h,M).
projection   Orthogonal projection onto the complement of the collision
             invariants in the M^{-1}-weighted inner product.
timestep     Classical RK4 for the spatially homogeneous linearized
             equation df/dt = L[f] (Sec. 4.2).
steady       The steady 1-D problem with diffuse walls (Sec. 5, Appendix B):
             upwind transport, residual with the binary operator, modified
             Newton operator, Newton iteration with tight GMRES solves.
learned      The fixed maps of the learned inner-solve correction (Hermite
             moments, features, correction field) and its tanh network with
             MSE gradient and Adam step.

Readings of the paper that the oracle takes where the text is silent or
inconsistent (each also implemented identically on the GPU side):
  R2  g-quadrature: Gauss-Jacobi-Radau in x = 2g/R - 1 with weight
      (1+x)^(4-2*omega), which absorbs g^2 B(g); fixed node g = 0;
      J = n/2 + 1 nodes (exact to degree n).  Alternative rule 1: weight
      (1+x)^2 with B(g_j) multiplied in.
  R3  gain constant: Phi_j(k) = 4 pi^2 W_j s_j(k) together with
      G = rho (pi theta)^(-3/2) exp(-|v|^2/theta).  Algorithm 1 prints
      32 pi^2, which with its own M^g normalisation gives a gain term
      8x too large (pinned by the Maxwell-molecule closed form
      L+[M] = 2 rho M in the tests).
  R4  phi_j = iDFT[sigma_j] where sigma_j doubles s_j at each Nyquist
      index (eq. (24) sums m over -N..N, so +N and -N coincide).
  R5  the product in eq. (24) is a plain cyclic convolution (no c_k
      halving of the Nyquist entries).
  R9  cutoff: r = h/M kept where M/rho >= eps, r = 0 otherwise; the
      loss term uses the uncut h.
  R17 diffuse walls: the wall density makes the discrete mass flux through
      the wall exactly zero (ghost rho_W E_W, E_W = exp(-|v-u_W|^2/(2
      theta_W)), rho_W from the outgoing half-range sum); the printed
      constants are its continuum limit.  The right wall reads the last
      cell (the printed formula names the first, a slip).
  R18 total mass: Q with Q^_0 = 0 in the residual, P L P in the Newton
      operator, and the initial guess and each iterate rescaled to the
      discrete mass C.
"""
