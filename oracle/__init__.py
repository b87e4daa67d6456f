"""Plain FP64 CPU oracle for the randomized two-site MPO-MPO fit.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call or link anything in this package; only the
test suite, the smoke check and the CPU-baseline leg of the benchmark use it.

Every function follows the paper (Foderà, Ritter, Shinaoka, von Delft,
"Parallelized contraction of tensor trains or matrix product operators")
step by step, with numpy/LAPACK as the only primitives and no blocking, fusion
or reordering beyond what the paper states.  Citations name the section,
equation, algorithm or table of the paper.

Modules
  philox  counter-based Gaussian test matrix (Sec. 3, Fig. rsvd (b1))
  mpo     dense expansion, naive product (Alg. 1), inner products, norms
  canon   site-canonical and inverse-canonical gauges (Sec. 2.3.1)
  fit     environments, 2-site updates (Alg. 3/4), RSVD (Sec. 3.1),
          serial fit (Alg. 5), even/odd inverse-gauge schedule (Sec. 4)
  grad    loss at frozen truncation bases and its gradient

Parity status: see each module header; every function listed there is pinned
by a ``-m "not gpu"`` test against something other than itself.
"""
