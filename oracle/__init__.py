"""Plain FP64 CPU oracle for the Kohn-Sham LOBPCG eigensolve.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The HIP library and
its Python binding never import it and share no code with it.

What it computes, and where the paper defines it:

* ``hamiltonian``: H psi = T psi + V_loc psi + sum_a sum_j b_aj D_aj b_aj^T psi,
  with the kinetic term T applied through a discrete Fourier transform (the
  SCF task list of the paper names FFT for the Laplacian and a separate
  nonlocal pseudopotential operator).  Here the transform is a naive
  separable per-axis DFT with n x n matrices, never an FFT.
* ``linalg``: the generalised Hermitian eigenproblem H X = lambda S X of the
  LOBPCG subspace, reduced by a Cholesky factor S = L L^H to the standard
  problem K Z = lambda Z with K = L^-1 H L^-H and Z = L^H X (Eq. 1), where
  K is formed by two triangular solves instead of a HEGST-type reduction
  (the paragraph after Eq. 1).  The standard problem is solved by cyclic
  complex Jacobi rotations.
* ``lobpcg``: the block iteration (Knyazev's LOBPCG, cited for the
  eigensolver in the SCF task list), Rayleigh-Ritz on [X, W, P].
* ``precond``: the Teter-Payne-Allan kinetic preconditioner.
* ``cnn``: a 3-layer periodic 3x3x3 convolutional network with its analytic
  backward pass.
* ``cg``: the projected conjugate-gradient solve that makes training pairs.
* ``scf``: the self-consistent loop around the eigensolve (density, the
  Hartree potential by the periodic Poisson equation, a local density
  approximation, linear mixing), the "Others" of the paper's SCF cost
  breakdown.
"""
