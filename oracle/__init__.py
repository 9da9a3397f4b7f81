"""CPU FP64 oracle for the Kronecker-product SVD / split Bregman path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package. Only the
test-suite, the smoke entry point and the CPU-baseline leg of the benchmark use
it. It shares no code with the HIP path: both sides only consume the seeded
inputs drawn by the ``workloads`` module.

Every function is written from the paper (Alsubhi & Renaut, arXiv 2410.00233)
in plain NumPy/LAPACK, in float64 unless a dtype is requested, with no
blocking, fusion or reordering beyond what the cited definition or algorithm
states. Each function cites the passage it follows.

Modules
-------
operator  blur matrix A, the rearrangement R(A), its entries, dense and
          structured products, exact Kronecker SVD (section 2.1, Theorem 12.3.1)
philox    Philox4x32-10 counter-based generator + Box-Muller normals (the one
          random source both sides implement from its published definition)
kpsvd     EGKB (Algorithm 1), RSVD (Algorithm 2), Rayleigh-Ritz refinement,
          Kronecker terms (eq. "KP approx")
sb        KP apply (eq. "KPAx"), regularization operator (eq. "deriv"), CGLS
          (Algorithm 5), split Bregman anisotropic/isotropic (Algorithms 3, 4)
metrics   RE, ISNR, SNR (section "Performance Metrics") and the Kronecker
          approximation error ||A - A_k||_F

Parity status: every function is pinned by ``tests/test_oracle_*.py`` except
the auto-k rule on the paper's own problems (IR Tools data not available):
"parity unpinned" for the paper's printed k = 5 / 8 / 16.
"""
