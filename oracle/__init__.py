"""FP64 CPU oracle for the RWG-discretised EFIE and its Calderon product.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or links
this package; only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline`
leg of `bench.py` may use it.  It shares no code, table or constant with the GPU
library: every definition here is written out again from the literature and
the paper, in plain numpy/scipy (and, for gradients, torch CPU autograd).

Conventions (paper, Sec. II, eq. 5): the time factor is e^{+j omega t}, so the
3-D free-space Green's function is G_k(R) = exp(-j k R) / (4 pi R).  Galerkin
matrices follow the paper's definition (O)_ij = (lambda_i, O lambda_j) of
Sec. III, with RWG functions as the lambda's in 3-D.

Modules
  rwg         mesh validation and RWG basis topology
  quadrature  7-point degree-5 triangle rule and subdivided reference rules
  singular    closed-form potential integrals over a flat triangle
  efie        near-pair classification, T_A / T_Phi / Z assembly, excitation,
              far field and RCS
  krylov      LU reference solve, CGS and COCG
  mie         Mie series for a PEC sphere
  calderon    barycentric refinement, Buffa-Christiansen functions, the mixed
              Gram matrix and the Calderon-preconditioned operator
  cfie        the 3-D Calderon-stabilized CFIE: the magnetic (MFIE) operator K
              tested with rotated BC functions, its Calderon product and the
              combination with the EFIE product (the 3-D reading of eq. 16)
  bie2d       the paper's own 2-D method: single, adjoint double and hypersingular
              layer operators with the Hankel kernel on a closed polygon, the TM
              CFIE of a PEC cylinder, its Calderon-stabilized form C_p (eq. 16),
              the circular counterpart, the randomized skeleton of their
              difference and the Woodbury inverse (eqs. 17-18); the PEC-cylinder
              series solution
"""
