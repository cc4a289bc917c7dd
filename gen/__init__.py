"""Seeded synthetic inputs for the energy-minimization RCG.

This package only *builds inputs*: the SPD operator A, the tentative
prolongation P0, the fine near-kernel basis B and its coarse counterpart B_c
(the data the method receives, Sec. 3 and Sec. 3.2 of the paper).  It holds
none of the method's arithmetic: no sparsity-pattern expansion, no
constraint projection, no conjugate-gradient step.  Both the CPU oracle and
the GPU path consume what is built here.

Workloads (all seeded, all synthetic):

* ``poisson2d_32``   -- 2D 5-point Poisson on a 32x32 grid, 2x2 aggregates.
* ``poisson3d_het96``-- 3D 7-point Poisson on 96^3 cells, k=exp(N(0,2^2)),
                         harmonic face averages, 3x3x3 aggregates.
* ``elasticity_q1_40``-- trilinear hexahedral elasticity on 40^3 elements,
                         log-normal Young's modulus, six rigid-body modes,
                         3x3x3 node aggregates with a local QR of B.
* ``rgg_batch``      -- 256 random-geometric-graph Laplacians (mean degree
                         14, shift 1e-3), greedy aggregation.
* ``poisson3d_ln32`` -- 3D 7-point Poisson on 32^3 cells, k=exp(N(0,1)),
                         2x2x2 aggregates, plus a fixed random vector e.
* ``node_grid2d``    -- a 2D nodal system with full node blocks (node sizes
                         other than 3, for tests of the node kernels).
* ``tiny``           -- small random problems for pinning tests.
* ``cf_*``           -- classical C/F settings (A, strength graph, C/F split,
                         near-kernel modes) for the tentative set-up, Alg. 1,
                         and the P = [W; I] form.
"""

from .problems import (  # noqa: F401
    EminInput,
    poisson2d_32,
    poisson3d_het96,
    poisson3d_ln32,
    elasticity_q1_40,
    rgg_batch,
    rgg_one,
    fd_poisson,
    tiny_problem,
    node_grid2d,
    by_name,
    CFInput,
    cf_poisson2d,
    cf_linear2d,
    cf_random,
)
