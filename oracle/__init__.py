"""CPU FP64 oracle for the multigrid-preconditioned CG solve of K(rho) u = f.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the GPU library.
"""
