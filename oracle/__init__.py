"""CPU oracle for the triangular-domain EDM library.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) imports, links or calls anything in this package.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark use it.

What lives here, each a plain and slow restatement of what the paper fixes
(Navarro & Hitschfeld, "Improving the GPU space of computation under
triangular domain problems"):

* ``maps``   -- exact-integer block map g(lambda) (Sec. II-A, Eq. (2) and its
  proof, Eqs. (3)-(9)), the no-diagonal variant (Eq. (10)), the coverage of
  every comparison strategy (BB, LTM, RB, REC, UTM; Sec. III-B) by brute-force
  enumeration, the wasted-block closed forms (Sec. II-A) and the improvement
  model (Sec. II-B, Eqs. (11)-(15)).
* ``edm``    -- FP64 Euclidean distance map (Sec. IV, Eq. (17)), its
  gradient, the stress loss, and the stated BF16 Gram error bound.
* ``c/``     -- the same EDM / gradient written as plain C loops in double
  precision (OpenMP over rows), used for large sampled comparisons and timed
  as the CPU baseline.  ``native`` loads it.

Every function is pinned by ``tests/test_oracle_*.py`` against values that
do not come from the oracle itself (worked examples in the paper, closed
forms, scipy/torch reductions, brute-force enumeration, finite differences).
"""
