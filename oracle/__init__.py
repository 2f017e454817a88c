"""FP64 CPU oracle for the thick-restart Lanczos method for Hermitian
J-symmetric matrices (TRLAN-JSYM, Ishikawa & Sogabe, arXiv:2001.07428).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP implementation; the
two meet only at the seeded input generators, which hold no arithmetic of the
method.

Modules
-------
jsym     the J-structure: J, partner vectors, block-form operators (dense and
         4D stencil), dense materialisation, brute-force spectra, and the
         Fourier closed form of the constant-link stencil.
trlan    Algorithms 1 and 2 of the paper, in plain complex128 NumPy.
casea    the paper's known-spectrum generator of Sec. 4.1 (Case A).

Every function is pinned by CPU tests against something other than itself
(brute-force diagonalisation, closed forms, the paper's invariants).
"""
