"""Plain FP64 CPU oracle for the HR DD NM-ROM (arXiv 2305.15163).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its Python
binding, the benchmark's timed leg) may import, call or link this package.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg use it.

The oracle shares no code with the GPU path.  It is written from the paper, in its
notation and order, with numpy/scipy primitives (sparse products, dense solves, SVD)
and no blocking or fusion beyond what the paper states:

  burgers.py         Section 7.1: exact solution, central-difference residual and Jacobian
                     in the Kronecker/matrix form of the paper, monolithic Newton FOM.
  ddmaps.py          Section 2: residual/interior/interface sampling, ports, A_i.
  autoencoder.py     Sections 3.4, 5.1, 7.3: banded masks, shallow sparse autoencoders,
                     hand-written gradients, Adam training.
  hyperreduction.py  Sections 3.3, 5.3-5.4: POD energy criterion, greedy collocation
                     sampling, subnet extraction.
  rom.py             Section 4: DD-LSPG objective with collocation HR under the weak
                     FOM-port or the strong ROM-port constraint, Lagrange-Gauss-Newton SQP
                     with a full dense KKT solve and Armijo backtracking; DD-FOM SQP;
                     relative error (eq. relative_error).
  srpc.py            Section 3.2: ports, port decoders, the implied interface decoders and
                     the linear ROM-port constraint.
  lsrom.py           Section 3.3: LS-ROM (affine or POD maps) with collocation or gappy-POD
                     HR, solved along routes independent of rom.py (null-space QP steps).
  proposal.py        learned initial-iterate proposal (forward/backward, Adam, FP64)
                     and the zero-start fallback rule.
  build_model.py     offline pipeline (snapshots -> autoencoders -> HR -> model pack).
  pack.py            model pack (.npz) -> ROMModel.

Parity unpinned: the greedy sampler (hyperreduction.greedy_sample) follows the cited
algorithm by reading only; it is pinned by invariants, not by values.
"""
