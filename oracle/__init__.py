"""FP64 CPU oracle for stochastic texture filtering (STF) with sample reuse.

TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or call this package. The product
path (the HIP library and its Python binding) never does, and this package
imports nothing from it.

The oracle is a plain, slow, step-by-step implementation of what the GPU path
computes, written from the paper (Wronski, Pharr, Akenine-Moeller, "Improved
Stochastic Texture Filtering Through Sample Reuse", 2025):

  * texel-space coordinates (Sec. 4.5 listing: uv * size - 0.5),
  * bilinear (Sec. S6, GetFilterPMF) and bicubic B-spline (Sec. 5.4) filter
    weights, which double as the sampling PMF (Sec. 4.2),
  * one-tap STF texel selection (Sec. 2.2, Sec. S1),
  * sharing footprints inside an 8x8 wave tile (Sec. 4.3),
  * the multi-PDF weighted importance sampling estimator, Eq. (14)
    (Sec. 4.2; loop structure of Sec. 4.5),
  * the deterministic filtered value, Eq. (3),
  * the adjoint of Eq. (14) with respect to the texels, and through the
    latent decoder MLP to the latents and the decoder's weights and biases.

footprint_oracle holds the sparse sharing-footprint generator (Sec. 4.3,
Sec. S5); its header lists the readings it takes.

Parity status: the counter-based hash (pcg4d) has no published test vectors
available offline; it is pinned by statistical properties only ("parity
unpinned" against its publication). Footprint placements 2x2w/3x3/4x4 follow
a documented reading because the paper's figures are unavailable ("parity
unpinned" against those figures). Everything else is pinned by tests under
tests/ that use closed forms, invariants and brute force.
"""
from .stf_oracle import *  # noqa: F401,F403
from .stf_oracle import __all__  # noqa: F401
from . import footprint_oracle  # noqa: F401,E402  (sparse footprint generator, Sec. S5)
from . import estimators_oracle  # noqa: F401,E402  (comparison estimators, Sec. 4.1)
