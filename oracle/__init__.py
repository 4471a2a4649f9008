"""Plain, slow FP64 CPU oracle for the ACP phonon method (test infrastructure).

This package is the checker, not the product.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the library and
its Python binding never do, and the oracle never imports them.  It shares no
code with the HIP path: the only common inputs are the seeded random draws of
``workload.seeds``.

Modules
  model   discrete model of Sec. 2.1 / Sec. 4.1: FD Laplacian, Yukawa operator,
          Gaussian pseudocharges, SCF ground state, energy, forces, local Hessian
          terms, frozen-phonon finite differences
  chi0    exact response: sum-over-states chi0 (Eq. (2.17)), Sternheimer form
          (Eq. (2.18), Alg. 1) with dense solves, dense Dyson (Eq. (2.14)),
          exact Hessian (Eq. (2.11))
  acp     the ACP method step by step (Alg. 2, 3, 4) with exactly solved
          shifted equations
  krylov  plain batched CG and MINRES for the projected shifted equations
"""
