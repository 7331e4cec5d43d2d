"""CPU oracle for parallel Graver-basis extraction (Liu, Wang, Yang,
"Parallel Graver Basis Extraction for Nonlinear Integer Optimization").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously
correct reference of what the GPU path computes.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does, and it shares no code, tables or helpers with the HIP
library (the only shared module is the seeded input generator, which holds
none of the method's arithmetic).

Modules and what they follow:

* ``lattice``   -- integer kernel basis B from a column-style Hermite normal
                   form (Lemma 3.1, Theorem 3.2), LLL reduction (Appendix A,
                   Algorithm 3), the coordinate map z = (B^T B)^-1 B^T g
                   (Section 3.1).
* ``surrogate`` -- the surrogate Phi and its gradient (eq. loss), Adam
                   (Section 3.2), and Parallel Extraction (Algorithm 2).
* ``conformal`` -- the conformal order, Graver basis by brute force in a
                   box (Section 1), exact kernel check (condition C1).
* ``minimal``   -- the minimality filter with deduplication (condition C3).
* ``augment``   -- the augmentation scheme (Algorithm 1) and objective.
* ``philox``    -- Philox4x32-10 counter-based generator (Salmon et al.,
                   SC'11), used to draw Uniform(l-u, u-l) start points.

Floating point is IEEE binary64 throughout, with every sum taken in a fixed
ascending order and no fused multiply-add, so the FP64 GPU path can be
compared bit for bit.  Integer results use exact Python / numpy integers.
"""
