"""CPU oracle for vectorized secure decision-forest inference (COPSE, PLDI'21).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or runs
anything here; only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark do.  The oracle shares no code, tables or constant generators
with the GPU path: primes, roots of unity, NTTs, base conversions and
samplers are written again here from their definitions.

Layout
  forest.py    plain forest evaluator: the definition of the result
  compiler.py  forest -> padded thresholds, reshuffle/level matrices, masks
  slotsim.py   Algorithm 1 on plaintext slot vectors mod t (exact layout)
  nt.py        number theory: primality, prime chains, roots of unity
  sampling.py  SHAKE-256 streams and the uniform/ternary/error samplers
  cbgv.c       plain C (unsigned __int128) ring kernels used by bgv.py
  bgv.py       BGV over an RNS chain: keys, encrypt/decrypt, ops
  circuit.py   the canonical encrypted schedule of Algorithm 1
"""
