"""CPU FP64 oracle for the Nedelec/Schwarz Maxwell solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
re-statement of what the GPU path computes, written from the paper's
equations (time-harmonic Maxwell problem, its variational form, the
scattering functional, the ORAS/GMRES solver and the inverse-problem cost).
Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the HIP path; both sides
only share the seeded input generators in the ``workload`` package.

Modules
  fem      topology, element matrices, global operator, sources, direct solve
  schwarz  partition, overlap, partition of unity, colouring, ORAS matrices
  krylov   right-preconditioned flexible GMRES
  gradient adjoint-state gradient of the regularised misfit
  learned  learned coarse-space correction (pooling, network, training target)

Parity status of each function is stated in its docstring ("pinned by ..."
or "parity unpinned").
"""
