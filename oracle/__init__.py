"""Oracle: plain, slow, CPU FP64 reference for the partitioned
shift-without-invert eigensolution and the transmission T(E).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package; only the test suite, the smoke check and the
CPU-baseline leg of the benchmark do.  It shares no code with the HIP library
(no kernels, headers, helpers or table generators); the only module both sides
use is `synth`, which draws the seeded workloads.

Each function cites the passage of Feldman & Zhou, "A partitioned
shift-without-invert algorithm to improve parallel eigensolution efficiency in
real-space electronic transport" (arXiv:1606.01139) that it follows.  Where the
paper is silent the reading used is stated at the function.

Modules:
  operator   -- the real-space operator A = H - i(Gamma_L + Gamma_R), Eq. (1)
  eigen      -- per-window eigenpairs nearest a real shift, Eq. (3)
  partition  -- Algorithm 1 (window counts and shifts), Algorithm 2 (combine)
  transport  -- T(E) = Tr{G Gamma_R G^dagger Gamma_L} (Section 1)
  gradient   -- derivative of sum_e T(E_e) w.r.t. V(r) and the absorber
                parameters (not in the paper; exact derivative of the
                quantity the pipeline computes)

Parity pins (tests/test_oracle_*.py) tie every function to something other
than itself: exact rational FD moments, closed-form spectra of the discrete
Laplacian, dense brute force, the trace identity, Eq. (5)'s bound, the dense
direct solve of G, and finite differences.
"""
