"""Plain FP64 CPU oracle for the far-field occupied exchange K^ff_ri of
occ-FMM-K (Le & Shiozaki, arXiv:1708.05353).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The HIP library never calls it and
shares no code with it: this package has its own solid harmonics (complex,
m = -l..l), its own AO multipole integrals (tensor-product Gauss-Hermite
quadrature), its own box tree and its own step-by-step FMM, all written from
the paper's equations in NumPy complex128 / float64.

Modules
  harmonics  scaled regular/irregular solid harmonics, Eq. (4a,b)
  basis      normalised Cartesian s/p primitives, pairs, AO multipoles, Eq. (8)
  tree       hierarchical boxes, neighbour and interaction lists (Theory section)
  fmm        MO transforms Eq. (15), M2M/M2L/L2L Eq. (17a-c), K^ff Eq. (18);
             direct ancestor-centred sum (same result, no translations)
  exact      s-type exact ERIs via the Boys F0 closed form; point-charge limit
  mlp        small MLP forward/backward/Adam in float64 (rank-selector oracle)
"""
