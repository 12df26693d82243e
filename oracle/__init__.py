"""FP64 CPU oracle for differentiable-ray-tracing radio calibration.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
implementation of what the calibration hot path computes, written from the
paper (Hoydis et al., "Learning Radio Environments by Differentiable Ray
Tracing", arXiv 2311.18558) in float64 / complex128 with plain PyTorch CPU
ops so that autograd supplies the reference gradients.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it; the GPU
library never calls into it and shares no code with it.

Modules
  em       constants, material transforms, permittivity, Fresnel, antenna bases
  trace    per-path field computation (transfer chain -> path coefficient)
  channel  array coefficients, CFR synthesis, CIR / power-delay profile, losses
  mlp      neural materials: positional encoding + MLP (FP64 and BF16-emulated)
  adam     the Adam update
  diffuse  Lambertian single-bounce diffuse interaction

Readings taken where the paper is silent are listed in the design notes and
restated in the docstring of the function that applies them.
"""
