"""MI355X-native SPAI-smoothed geometric multigrid (He, Liu and Wang,
arXiv 2206.05543): V(1,1) and W(1,0) cycles for the 2D 5-point and 3D
7-point Dirichlet Laplacian with the optimised sparse-approximate-inverse
smoothers (and the wider 19-/27-point 3D stencils), as gfx950
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
# The wider 3D stencils the closing remark of Section 3.2 mentions (centre,
# faces, edges[, corners]; damping folded in): the minimax optima of the
# smoothing factor over the 19- and 27-point symmetric families, mu = 0.2266
# and 0.1970 against 25/73 = 0.3425 for M7, from a numerical minimax search
# over the sampled symbol (the paper gives no closed form for them).
M19 = (0.20341196152997898, 0.03826561652493997, 0.007552424314552823)
M27 = (0.19656718416287874, 0.03973166487560058, 0.011501271415304574, 0.003659495448695544)

# The smoothers compared in Section 4 (2D: Jacobi, the 5-point stencils of
# Tang-Wan and of Section 3.1, additive Vanka, M9; 3D: Jacobi, M7), and in 3D
# the wider M19 and M27.
SMOOTHERS = {
    2: {"J": JACOBI_2D, "TW5": TW5, "M5": M5, "Vanka": VANKA, "M9": M9},
    3: {"J": JACOBI_3D, "M7": M7, "M19": M19, "M27": M27},
}


def paper_coeffs(d):
    return M9 if d == 2 else M7
