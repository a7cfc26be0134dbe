"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never calls it, and the oracle imports nothing from the product.
It shares no code with the GPU path; the only common dependency is the seeded
input description in `synth` (circuits as explicit FP64 gate lists, bitstring
batches), which holds none of the method's arithmetic.

Modules:
  network   the tensor network of a circuit (gate fusion, folded kets, legs),
            written from the network convention the library documents.
  statevec  O1: dense FP64 state-vector simulation, amp(s) = psi[s].
  tn        O2: naive FP64 pairwise contraction of the network with output
            and sliced legs fixed, in the oracle's own greedy order.
  xeb       O3: linear XEB (Eq. 1) with exactly rounded sums.
  memo      O4: distinct-key counts per tree node (Appendix C) and a direct
            run of the eval_all / eval' procedure (Algorithms 3 and 4) on
            symbolic values, counting the pairwise contractions it performs.

Every function states the passage it follows.  Pins live in tests/ (marker
"not gpu").  Precision: FP64 throughout (complex128).
"""
