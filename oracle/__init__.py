"""Plain FP64 CPU oracle for the FFT-PIM periodic superposition sum.

This package is test infrastructure.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import it; the product library never
does, and it imports nothing from the product library.

Modules
-------
pgf      periodic Green's function G^p (Sec. 2: Eq. (2), the spectral series
         Eq. (pgf), the neutral static series Eq. (lgf)), with textbook Ewald
         splittings as the fallback where the paper's series converge slowly.
psp      the periodic scalar potential, Eq. (1), as a direct pair sum, and its
         conjugate transpose.
steps    the FFT-PIM algorithm of Sec. 3 written step by step (far zone
         Steps 1-3, near zone Steps 1-4), used to pin the GPU kernels to
         rounding level independently of the method's approximation error.
"""
