"""MI355X-native Quadrature-to-Expansion (Q2X): Laplace multipole coefficients
of flat triangles (single and double layer), segments and tetrahedra about
their leaf-box centres, computed with the O(1)-per-moment recursions of
Gumerov, Kaneko & Duraiswami (arXiv 2107.10942) in hand-written HIP kernels
for gfx950 behind a C ABI (include/q2x.h)."""
from . import q2x  # noqa: F401
