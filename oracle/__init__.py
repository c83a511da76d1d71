"""Slow, plain CPU oracle for the random-circuit-sampling hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python
binding imports, calls or links anything in this package; only the tests,
the smoke check and the CPU-baseline leg of the benchmark do.  The oracle
shares no code with the HIP path: it re-derives every step from the
definitions (the circuit family of the paper's Section 3.1, the state /
sample / score pipeline of Section 3.2, linear XEB of Section 5.1) in plain
numpy complex128 (fp64), with library routines (matmul, QR, SVD) used only
as single steps.

Modules
  philox     Philox4x32-10 counter-based generator (Salmon et al., SC'11)
  circuit    grid, couplers, gate set, gate draws (Section 3.1 circuits)
  dense      dense state-vector simulator, n <= 28
  mps        plain snake-ordered MPS with SVD truncation (same schedule)
  sample     sequential conditional sampler, amplitudes, linear XEB
  precision  exact bfloat16 round-to-nearest-even emulation, split-bf16
  rsvd       randomized truncated SVD (Halko-Martinsson-Tropp 2011)
  mlp        rank-prediction MLP, fp64 forward/backward and Adam
"""
