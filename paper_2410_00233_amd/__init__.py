"""MI355X-native Kronecker-product SVD and split Bregman deblurring.

Implements the hot path of Alsubhi & Renaut (arXiv 2410.00233): the truncated
SVD of the rearranged blur R(A) by enlarged Golub-Kahan bidiagonalization
(Algorithm 1) and randomized SVD (Algorithm 2), the Kronecker-sum apply
(eq. "KPAx") and split Bregman TV deblurring with CGLS inner solves
(Algorithms 3-5), as hand-written HIP kernels for gfx950 behind the C ABI in
include/kpsb.h. ``api`` is the thin Python binding; ``build`` compiles the
library in-tree.
"""

__all__ = ["api", "build", "flops"]
