"""Plain FP64 CPU oracle of one Neu-PiG optimization step.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.
The product path (the HIP library and its Python binding) never does, and
shares no code, header, table or constant generator with it.

Everything is numpy (scipy for the DCT), float64, written to be read against
the paper section by section; no blocking, fusion or reordering beyond what
the definitions state (the Chamfer brute force is evaluated in vertex blocks
only to bound memory). Inputs arrive as float32 arrays and are promoted.

Parity status of each function (pins live in tests/test_oracle_*.py):
  grid_coords / trilinear / encode ...... pinned (affine reproduction, node
                                           values, weight partition of unity)
  time_code .............................. pinned (closed forms)
  mlp_forward / mlp_backward ............. pinned (torch.nn float64, FD)
  rodrigues / transform .................. pinned (scipy Rotation, invariants,
                                           known rigid motion)
  chamfer ................................ pinned (double-loop brute force,
                                           cKDTree distances, closed forms)
  confidence / loss ...................... pinned (hand-worked example,
                                           invariants)
  backward (all blocks) .................. pinned (central finite differences,
                                           torch autograd float64)
  precond_dct / precond_cg ............... pinned (dense solve, lambda = 0
                                           identity, linearity, symmetry,
                                           constant preservation, mode scaling)
  adam ................................... pinned (closed-form first step,
                                           torch.optim.Adam float64)
  the robust Chamfer variant the paper cites from DynoSurf is not defined
  in the paper and is not implemented: parity unpinned.
"""
from .neupig import *  # noqa: F401,F403
