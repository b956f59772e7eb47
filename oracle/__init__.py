"""FP64 CPU oracle of the sparse FFT hot path (Hassanieh, Indyk, Katabi, Price,
"Nearly Optimal Sparse Fourier Transform").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of the paper's method in numpy float64.  It exists to
check the HIP library against.  Only the test suite, the smoke entry point and
the benchmark's CPU-baseline leg may import it; the product path never does.

It shares no code with the HIP library (no headers, helpers, tables or
generated constants).  The only thing both sides consume in common is the
seeded input signal built by ``siggen``, which holds none of the method's
arithmetic.

Modules
-------
fft       naive O(n^2) DFT and an own radix-2 FFT (Section 2 convention)
window    flat window G and its ideal spectrum G' (Section 7 construction)
rng       SplitMix64 in counter form and the per-hashing draws
hashing   permutation, bin/offset maps, HashToBins (Algorithm 1; HashToBins lemma of Section 3)
exact     exactly sparse recovery (Algorithm 1, NoiselessSparseFFT)
general   general recovery (Algorithms 2 and 3, SparseFFT/LocateSignal/...)
metrics   Err(x, k) and the l2/l2 ratio (Section 1 eq. (1), Section 4.2)

Parity status: every function is pinned by a CPU test in ``tests/`` against a
closed form, an invariant or brute force, except the noisy general-mode
location/estimation outcome, which is "parity unpinned" beyond the l2/l2
statistical guarantee (see ``general.py``).
"""
