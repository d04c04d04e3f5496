"""Plain FP64 CPU oracle for the fPEPS boundary-MPS row absorption.

TEST INFRASTRUCTURE ONLY. This package exists to check the device library:
only the tests, the smoke check and the benchmark's CPU-baseline leg may
import or run it. The product path never calls it, and it shares no code
with the device library (only the seeded input generators of ``workloads``).

Modules: rng (Philox4x32-10, SplitMix64, Box-Muller), blocks (dict-of-blocks
contraction), chain (the implicit site operator and its transpose), rsvd
(randomized SVD, Halko et al. Example 1.6), zipup (row absorption),
expect (network value), exact (state-vector pins), cbe (controlled bond
expansion), flops (algorithmic flop count), heff (the effective single-site
operator of the Davidson step).
"""
