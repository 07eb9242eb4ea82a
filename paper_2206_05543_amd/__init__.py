"""MI355X-native SPAI-smoothed geometric multigrid (He, Liu and Wang,
arXiv 2206.05543): V(1,1) cycles for the 2D 5-point and 3D 7-point Dirichlet
Laplacian with the optimised sparse-approximate-inverse smoothers, as gfx950
HIP kernels behind the C ABI of include/spaimg.h.

Importing the package loads nothing; ``paper_2206_05543_amd._lib`` binds the
library on first use (``_lib.lib()``, ``_lib.Multigrid``) and fails loudly if
it is not built.
"""
import math

# Smoother coefficients (h-free, damping folded in): see include/spaimg.h.
OMEGA_M9 = (309.0 - 12.0 * math.sqrt(10.0)) / 1720.0     # Theorem 3.1
M9 = tuple(OMEGA_M9 * w / 24.0 for w in (44.0, 10.0, 3.0))
M7 = (16.0 / 73.0, 2.0 / 73.0)                           # Theorem 3.2
JACOBI_2D = (0.2, 0.0, 0.0)
JACOBI_3D = (1.0 / 7.0, 0.0)
M5 = (12.0 / 41.0, 2.0 / 41.0, 0.0)
VANKA = (0.28, 0.04, 0.01)
TW5 = (17.0 / 61.0, 3.0 / 61.0, 0.0)

# The smoothers compared in Section 4 (2D: Jacobi, the 5-point stencils of
# Tang-Wan and of Section 3.1, additive Vanka, M9; 3D: Jacobi, M7).
SMOOTHERS = {
    2: {"J": JACOBI_2D, "TW5": TW5, "M5": M5, "Vanka": VANKA, "M9": M9},
    3: {"J": JACOBI_3D, "M7": M7},
}


def paper_coeffs(d):
    return M9 if d == 2 else M7
