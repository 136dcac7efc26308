"""FP64 CPU oracle for the edge-alignment cost, its SE(3) pose gradient and the
pose update of EPO (edge-based pose optimization).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package.  It
shares no code with the HIP path (no kernels, headers, helpers or constant
tables) and imports nothing from it; both sides consume the same seeded inputs
from the separate input generator.

Everything is plain NumPy in float64 (the distance transform in exact
integers), written from the paper's definitions:
  edt.py       exact squared Euclidean distance transform (DTF, Sec. 3):
               brute force, Felzenszwalb-Huttenlocher, separable min-plus
  geometry.py  SE(3) exponential / logarithm, left perturbations
  cost.py      lift -> world -> target camera -> pinhole projection ->
               bilinear DTF sample -> clamp -> Huber (Eqs. pi, L, L_ij, d_ij;
               Alg. 3), per-direction mean over valid residuals, loss and the
               analytic left-twist pose gradient; frozen-branch evaluation for
               finite differences
  loop.py      clamp annealing, learning-rate warm-up + cosine (Sec. 4
               implementation details, Alg. 3), Adam on se(3) twists, the
               iteration loop
  convergence.py  pose-change signal theta_95 and the dual-phase windowed
               convergence test (Sec. 3 optimization schedule, Alg. 2)
  joint.py     the joint phase's AdamW step of focal scales and per-pixel
               depth scale and shift, gated by the convergence phase
  mlp.py       the paper's pose refiner: MLP, 6D rotation and Gram-Schmidt,
               translation offset, AdamW, with BF16 operand rounding
  sampling.py  per-step stochastic image-pair sub-sampling (SplitMix64 draws)
  viewgraph.py cycle-consistent reprojection test for candidate image pairs

Parity status of each function is stated in its module header.
"""
from . import edt, geometry, cost, loop  # noqa: F401
