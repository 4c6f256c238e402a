"""Test oracle for the leaf-box reduction of the two-level HPS solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
implementation written from the paper (Kump, Yesypenko, Martinsson, "A
Two-Level Direct Solver for the Hierarchical Poincare-Steklov Method").  Only
the test suite, the smoke check in __graft_entry__ and the CPU-baseline leg of
bench.py may import it.  The solver package never imports it and shares no
code with it; the two meet only through the seeded inputs in ``workloads``.

Modules
  cheb       Chebyshev-Gauss-Lobatto nodes and the spectral differentiation
             matrix (Sec. 2.1).
  leaf       local collocation blocks A_ii, A_ib, A_bi, A_bb of one box
             (Sec. 2.1 eq. Aentries, Sec. 2.2 eq. blocksys1) and the per-box
             reduction: solution operator S, DtN map T, equivalent load g
             (Sec. 2.2 definitions of S and T, Sec. 3.1 eq. t-block).
  interface  global face numbering, assembly of the sparse interface system,
             its sparse LU solve, and interior reconstruction (Alg. 1, Alg. 2).
  brute      the global collocation system of eq. Aentries formed densely and
             solved directly (the pin for the static condensation).
  adjoint    gradient of a data misfit with respect to b through transposed
             solves of the factorization in eq. factor2.
  parabolic  Crank-Nicolson time stepping (Sec. 4.4) of u_t = nu Lap u +
             kappa^2 b u on the global collocation system of brute.

Parity status: every function here is pinned by tests/test_oracle_*.py
against closed forms, polynomial exactness, invariants, manufactured
solutions or the brute-force global solve, except the LU pivot sequence,
which is parity unpinned by design (factors are not unique and are never
compared).
"""
