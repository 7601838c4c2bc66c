"""FP64 CPU oracle for the SEM pressure-Poisson hot path.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import or call anything in this package. The product path
(the HIP library and its Python binding) never routes through it, and the two
share no code: this package imports neither the library nor its binding, and
computes every quantity (Gauss-Lobatto points, derivative and interpolation
matrices, geometric factors, Ax, gather-scatter, Jacobi, Chebyshev, the V-cycle,
PCG and flexible CG) from its own plain NumPy/SciPy code.

What is computed follows arXiv 2110.01716 (NekRS on Summit):
  * SEM basis on GLL points and tensor contractions: Algorithms, eq. field1
    and its footnote on the derivative matrix;
  * p-multigrid with tensor-product interpolation and Chebyshev-accelerated
    Jacobi smoothing, all pMG steps in 32-bit: Implementation (pMG paragraph);
  * flexible CG around the pMG preconditioner: Implementation (FlexCG/GMRES
    paragraph); Jacobi-PCG: Implementation (Helmholtz paragraph);
  * gather-scatter as exchange-and-sum of shared values keyed by global IDs:
    Implementation (Autotuned Communication).
Where the paper leaves a step unstated, the textbook SEM definition is used
(the readings are listed in the design notes of the repository).

Modules:
  reference_ops  GLL nodes/weights, derivative and interpolation matrices
  operators      geometry, local Ax, gather-scatter, mask, diagonal, assembly
  solvers        PCG, flexible CG, Chebyshev smoother, power iteration
  pmg            coarse levels and the V-cycle
  counter_rng    splitmix64 start vectors
"""
