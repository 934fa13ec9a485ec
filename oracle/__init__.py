"""Plain FP64 CPU oracle of the inverse fast multipole method (IFMM).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code, table or
helper with the HIP library; both sides see the same seeded inputs from
``workloads.py`` and nothing else.

Every function cites the passage of Coulier, Pouransari & Darve,
"The inverse fast multipole method" (arXiv 1508.01835) that it follows. Where
the paper is silent or ambiguous, each module's header states the reading it
takes.

Modules:
  tree       cluster tree, neighbour/interaction/children lists, colours
  kernels    matrix-entry kernels K(r)
  chebyshev  Chebyshev nodes and Lagrange interpolation
  h2         the H2 (black-box FMM) representation R1, its matvec, dense form
  extended   extended sparse system E: orthonormal bases, weights, sigma_0
  ifmm       level-by-level elimination with fill compression, merge, solve
  gmres      right-preconditioned (flexible) and left-preconditioned GMRES
  graph      generic block elimination on the graph of a block system
"""
