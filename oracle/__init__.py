"""CPU oracle for FNT-based Reed-Solomon erasure coding over GF(65537).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the coding path computes, written from Soro & Lacan,
"FNT-based Reed-Solomon Erasure Codes".  Only the test-suite, the smoke run
and the benchmark's CPU-baseline leg may import it; the product path never
routes through it and shares no code with it.

All arithmetic is exact integer arithmetic modulo p = 65537 on Python ints or
numpy int64 arrays.  Each function cites the section / equation it follows.

Modules:
  field     -- the prime field, primitive root 3 and the n-th roots (Sec. II-A/B)
  transform -- the DFT over GF(p) by definition and by divide and conquer (Sec. II-A)
  poly      -- polynomial product, derivative, evaluation (Sec. II-B)
  codec     -- encoder (Sec. II-B), decoders by Gaussian elimination and by
               Lagrange interpolation (Sec. II-B), locator quantities used by
               the six-step interpolation (Sec. II-B, steps 1-6)
  direct    -- the quadratic encoders and decoders of Sec. III (Tables I and II,
               and the classic quadratic schemes of its footnote)
  chirp     -- evaluation on a geometric sequence by one middle product
               (Sec. II-B, steps 3 and 5; Sec. III)
"""
