"""MI355X-native inversion-based triangular solve (L X = B).

The solve follows the paper's method: the n0 x n0 diagonal blocks of L are
inverted by recursive triangular inversion (Alg. RecTriInv inside Alg.
Diagonal-Inverter), then a blocked forward sweep of dense matrix products
(Alg. It-Inv-TRSM) computes X.  All arithmetic runs in hand-written HIP
kernels for gfx950 behind the C ABI declared in ``include/trsm.h``; this
package only marshals arguments (``paper_1612_01855_amd.trsm``) and draws
seeded inputs (``paper_1612_01855_amd.inputs``).

Importing the package does not load the GPU library; ``trsm`` does, and it
raises if the library has not been built.
"""

__all__ = ["inputs", "trsm"]
