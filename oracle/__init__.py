"""FP64 CPU oracle for the BTTB gravity/magnetic operators and the joint RRCG solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
no code with the GPU path.

Everything here is plain, slow and written to be checked against the paper
(Vatankhah, Renaut, Huang, Mickus, Gharloghi, "Large-scale focusing joint inversion
of gravity and magnetic data with Gramian constraint", arXiv:2112.15562) by eye:

* ``prism``     -- closed-form prism kernels (Sec. 2.1, eq. d=gm) and the dense
                   sensitivity matrix built entry by entry from absolute coordinates.
* ``bttb``      -- the kernel array T of Sec. 2.7.1 and the FFT2 products
                   (forward: IFFT2(FFT2(T) . FFT2(X)); transpose: with conj(FFT2(T))),
                   plus the weighted products of eq. (matrixvector).
* ``rrcg``      -- the Gramian (eq. Gramian), its ascent directions (eqs. RRCG:2-3,
                   steepestascenta/b), the L1 weight (eq. WL) and the RRCG iteration
                   (eqs. RRCG:1-8, Sec. 2.5 bounds, Sec. 2.6 chi^2, eq. regpara).
* ``dft``       -- brute-force O(N^2) DFTs used to pin FFT kernels.

Parity status of each function is stated in its module header.
"""
