"""FP64 CPU oracle for CAV-multigrid-preconditioned FGMRES (test infrastructure).

This package is test infrastructure. Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does.
It shares no code with the GPU library: it takes its inputs from `workloads`
and computes everything else itself with numpy/scipy in float64.

What it computes, module by module (paper sections in brackets):
  mac        periodic MAC grid D, G, L, A0 and the reduced operator K_E      [Sec. 2, Eq. intro_saddle]
  ib         4-point kernel, interpolation J, spreading S, force laws E,
             Eulerian elasticity E_E = S E J                                 [Sec. 2, Eq. disc_force_law, Sec. 5.2, App. A]
  hierarchy  RT0 / bilinear transfers, Galerkin coarse E_E                  [Sec. 4]
  patches    standard Vanka, box B(b,o) and CAV patch families              [Sec. 3.1-3.2, Eq. cav_patch_set]
  smoothers  equilibrated local solves, weighted additive and
             multiplicative Schwarz sweeps                                   [Sec. 3.3, Eq. additive_cav_saddle]
  multigrid  V(1,1) cycle with a bordered direct coarse solve               [Sec. 4]
  krylov     right-preconditioned FGMRES (CGS2, Givens)                      [Sec. 5]
  direct     bordered sparse LU reference solution                           [Sec. 2, Sec. 5.1 gauge mode]
  learned    small periodic conv net forward/backward (float64 reference)

Readings of the paper where it is silent are listed in the design notes and
repeated in the docstring of the function that takes them.
Parity unpinned: the iteration counts of the *additive* smoother have no
printed value in the paper; they are pinned only GPU-against-oracle.
"""
