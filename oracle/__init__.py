"""FP64 CPU oracle for the PMMM far field -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.
The HIP product path never touches it and shares no code with it.

Modules
  harmonics   solid harmonics R_l^m, S_l^m and their real storage (App. A)
  pmmm        literal FP64 PMMM: cells, P2M, transfer kernels, FFT
              convolution with the real-matrix M2L, periodic corrections,
              L2P with the order-1 L2L gradient (Sec. 2.1, App. A-C)
  exact       exact references: direct O(N^2) sum, Ewald sum, near field
  expansions  single-centre transformations (P2M, M2P, M2L, L2P, L2L, M2M)
              of App. A.3 in complex form, used to pin the mesh pipeline
  storage     per-order fixed-point coefficient records (Sec. 5.3) and the
              complex composition of two real sets (App. D)
  hierarchical  the two-level PMMM of Sec. 5.2: coarse PMMM plus the fine
              level for the pairs whose coarse cells are near

Parity status: every function listed above is pinned by a CPU test under
tests/test_oracle_*.py against values fixed by the paper (Table RSlm), by
textbook mathematics (associated Legendre functions, Laplace's equation,
addition theorems, the rock-salt Madelung constant, the bit counts of
Sec. 5.3) or by brute force.
"""
