"""Plain FP64 CPU oracle for the Gaussian-mixture SMC move stage.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import or call this package; only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code with
the GPU path: every function here is written from the paper's definitions
(arXiv 2503.16028, "Sequential Monte Carlo with Gaussian Mixture Approximation
for Infinite-Dimensional Statistical Inverse Problems") in NumPy/SciPy, float64,
without blocking, fusion or reordering beyond what each definition states.

Modules
  philox     Philox4x32-10 counter RNG (Salmon et al., SC'11) and the draw layout
  problem    problem definition: grids, KL eigenpairs, observation nodes, data
  forward    Darcy forward map by sparse direct solve (Sec. 3.2, eq. (example2:PDE))
  moves      pCN, pCN-GM (Sec. 2.3, Alg. 2) and pCN-Langevin moves, MH acceptance
  temper     ESS bisection of the next temperature (App. C)
  resample   systematic resampling with an exact integer CDF (Alg. 1, resampling)
  gmfit      diagonal Gaussian-mixture EM with k-means++ seeding (the stage input)
  smc        the SMC loop of Alg. 1 with the pCN-GM mutation (SMC-pCN-GM) and SMC-GM (Alg. 3)
  adjoint    gradient of the potential by an adjoint solve
  example1   the paper's multi-modal L^2 example (Sec. 3.1) and its exact mixture posterior
  linear     closed-form linear-Gaussian posterior (test target)
  quadrature brute-force posterior moments for tiny problems (test target)
"""
