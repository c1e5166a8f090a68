"""CPU oracle for the Winograd (Toom-Cook) layer with arbitrary points.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything in this package.
Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.

The oracle is written from the paper (arXiv:2201.10369) and is deliberately
plain: exact rational arithmetic for the construction of the transform
matrices (Section 4.1 and the modified form with the point at infinity,
Section 4.2), explicit fixed-order float32 loops for the Winograd evaluation
(eq. conv_1d and the nested 2D form eq. conv_2d), float64 direct convolution
(eq. conv) for the reference, and the L1 error metric of Section 6.

Modules
-------
toomcook : exact construction, point families (Section 5), exact tiles/layers
fp       : float32 / float16 / bfloat16 Winograd tiles and layers, float64 and
           float32 direct convolution, error metrics
sweep    : the error sweep over c (Section 6.1 / 6.3)
mlp      : float64 reference of the surrogate network, its gradient and Adam

Every function in here is pinned by tests against values or facts that do not
come from the oracle itself (printed matrices and tables of the paper, exact
identities, brute force, library routines); where no such pin exists the
function's docstring says "parity unpinned".
"""
