"""FP64 CPU oracle for the separated-operator apply on Legendre multiwavelet trees.

This package is TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The product library
(the HIP path behind the C ABI) never imports, links or executes anything here,
and nothing here imports the product package.

Every function is a plain, unblocked restatement of the mathematics of the
paper (arXiv:1507.01888, "MADNESS: a multiresolution, adaptive numerical
environment for scientific simulation"), Section 2:

* basis      -- scaling functions, eq. (scalingfunc), and the two-scale filter
                that connects levels n and n+1 (Sec. 2.1-2.2);
* projection -- orthogonal projection, eq. (projection), and adaptive
                refinement by comparing levels n and n+1 (Sec. 2.1);
* fit        -- Gaussian-sum representation of 1/r by trapezoidal quadrature
                of the integral identity in Sec. 2.3, and its bound-state
                Helmholtz analogue (kernel of eq. (bshkernel));
* blocks     -- 1D operator blocks of one Gaussian term (translation invariant,
                Toeplitz, Sec. 2.2) and their non-standard children blocks;
* apply      -- standard-form apply (level-n operator T^n = P^n T P^n) and the
                non-standard telescoped apply T^n = T^0 + sum_m (A^m+B^m+C^m),
                Sec. 2.2, with norm screening; sum-down reconstruction;
* tree       -- function trees, norm2 / trace / inner (Sec. 3.1 example);
* compress   -- wavelet (compressed) form, reconstruction and truncation (Sec. 2.2 fast
                wavelet transform);
* analytic   -- closed forms used as pins (Gaussian charge potentials).

Readings of points the paper leaves open are stated where they are used.
Parity of the mixed-precision tiers beyond the FP64 result is unpinned.
"""
