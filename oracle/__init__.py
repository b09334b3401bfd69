"""CPU oracle for the sparsifying preconditioner (Ying, arXiv:1409.0297).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it exists so that the tests, the smoke check and the
benchmark's CPU baseline can check the GPU library against an independent,
plain FP64 implementation written from the paper.  It shares no code,
tables or constants with the HIP library; the only common module is
``workloads`` (seeded input generators, no method arithmetic).

Layout
  spectral  -- shift/potential split (eq. Dsq), grids J and K, the unitary
               DFT as dense per-axis matrices, L (eq. Lsq), G (eq. G).
  stencil   -- leaf set partition, gamma/beta neighbourhoods, T_S by an
               explicit pseudoinverse (eq. Qc and Section 2.3), Q, C, P.
  nested    -- nested-dissection block elimination of the sparse P
               (Section 2.3, Figure 1) and its forward/back solve.
  gmres     -- right-preconditioned (flexible) GMRES with modified
               Gram-Schmidt and complex Givens rotations.
  pipeline  -- setup/solve wrappers and the dense ground truth.
"""
